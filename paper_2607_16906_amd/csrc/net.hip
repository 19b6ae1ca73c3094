// U-Net neural operator (Section 3.1, eq. (7), eq. (9)): handle, parameter
// repacking and the forward pass used as the flexible preconditioner.
//
// Architecture (the 3x3 / ReLU / doubling-channel reading of the paper's
// encoder-decoder): level l = 0..L-1 of the encoder applies two 3x3
// convolutions with ReLU (C 2^l channels), followed by a 2x2 average pool
// except at the last level; the decoder, from level L-2 down to 0, upsamples
// with a 2x2 stride-2 transposed convolution, concatenates the encoder output
// of the same level (encoder channels first) and applies two 3x3 convolutions
// with ReLU; a 1x1 head yields (Re, Im). The input field v is scaled by
// s = ||v|| / sqrt(n) before the network and the output is multiplied by s.
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "krylov.h"
#include "net.h"
#include "net_impl.h"
#include "net_kernels.h"

namespace hz {

static bool build_layers(const no_arch* a, std::vector<Layer>& L, int64_t& nparam, int64_t& pk, int64_t& nb) {
    if (!a || (a->in_ch != 2 && a->in_ch != 5)) return false;
    if (a->kind == NO_ARCH_UNET3) {
        if (a->levels < 1 || a->levels > 6 || a->base < 8 || a->base % 8) return false;
    } else if (a->kind == NO_ARCH_PAPER8) {
        if (a->levels < 1 || a->levels > 5 || a->base != 32) return false;
    } else {
        return false;
    }
    L.clear();
    nparam = pk = nb = 0;
    auto add = [&](int kind, int cin, int cout, int cin_p, int cout_p, int cat_c = 0, int cat_cp = 0) {
        Layer y;
        y.kind = kind;
        y.cat_c = cat_c;
        y.cat_cp = cat_cp;
        y.cin = cin;
        y.cout = cout;
        y.cin_p = cin_p;
        y.cout_p = cout_p;
        const bool k8 = kind == L_DOWN8 || kind == L_UP8;
        const int taps = kind == L_CONV3 ? 9 : (kind == L_CONVT2 ? 4 : (k8 ? 64 : 1));
        y.w_off = nparam;
        nparam += (int64_t)taps * cin * cout;
        y.b_off = nparam;
        nparam += cout;
        if (k8) y.a_off = nparam++;   // PReLU slope
        y.pk_off = pk;
        y.pk_len = (int64_t)taps * cout_p * cin_p;
        pk += (y.pk_len + 63) / 64 * 64;
        y.bias_off = nb;
        nb += (cout_p + (k8 ? 1 : 0) + 63) / 64 * 64;
        L.push_back(y);
    };
    const int lv = a->levels;
    if (a->kind == NO_ARCH_PAPER8) {
        // Table 2's layers: lv stride-2 8x8 convolutions down, lv transposed ones up (the decoder
        // input concatenates the encoder output of that size, encoder part first), 1x1 head
        const int c = a->base;
        add(L_DOWN8, a->in_ch, c, 8, c);
        for (int l = 1; l < lv; ++l) add(L_DOWN8, c, c, c, c);
        add(L_UP8, c, c, c, c);
        for (int l = lv - 2; l >= 0; --l) add(L_UP8, 2 * c, c, 2 * c, c, c, c);
        add(L_CONV1, c, 2, c, 16);
        return true;
    }
    int cin = a->in_ch, cin_p = 8;
    for (int l = 0; l < lv; ++l) {
        const int c = a->base << l, cp = round16(c);
        add(L_CONV3, cin, c, cin_p, cp);
        add(L_CONV3, c, c, cp, cp);
        cin = c;
        cin_p = cp;
    }
    for (int l = lv - 2; l >= 0; --l) {
        const int c = a->base << l, cp = round16(c);
        const int cu = a->base << (l + 1), cup = round16(cu);
        add(L_CONVT2, cu, c, cup, cp);
        add(L_CONV3, 2 * c, c, 2 * cp, cp, c, cp);
        add(L_CONV3, c, c, cp, cp);
    }
    add(L_CONV1, a->base, 2, round16(a->base), 16);
    return true;
}

// Repack one layer from the flat FP32 vector into [tap][cout_p][cin_p] (channels
// padded with zeros) in BF16, FP32 and FP64, and its bias into FP32 and FP64.
// The data-gradient packs hold the same values at [8 - tap][ci][co] (3x3) or [tap][ci][co]
// (transposed 2x2 and the 8x8 layers).
// One launch covers every layer: the blocks of layer l are [start[l], start[l + 1]).
__global__ void k_repack(const float* __restrict__ theta, const Layer* __restrict__ layers,
                         const int64_t* __restrict__ start, int nl, bf16_t* __restrict__ wb,
                         float* __restrict__ wf, double* __restrict__ wd, float* __restrict__ bf,
                         double* __restrict__ bd, bf16_t* __restrict__ tb, float* __restrict__ tf,
                         double* __restrict__ td) {
    int l = 0;
    while (l + 1 < nl && (int64_t)blockIdx.x >= start[l + 1]) ++l;
    const Layer ly = layers[l];
    const int64_t idx = ((int64_t)blockIdx.x - start[l]) * blockDim.x + threadIdx.x;
    if (idx < ly.pk_len) {
        const int cis = (int)(idx % ly.cin_p);      // stored input channel
        const int64_t r = idx / ly.cin_p;
        const int co = (int)(r % ly.cout_p);
        const int tap = (int)(r / ly.cout_p);
        // logical input channel; a concatenated input keeps each part's padding
        int ci = cis;
        bool live = cis < ly.cin;
        if (ly.cat_cp > 0) {
            if (cis < ly.cat_cp) {
                live = cis < ly.cat_c;
            } else {
                ci = ly.cat_c + (cis - ly.cat_cp);
                live = ci < ly.cin;
            }
        }
        float v = 0.0f;
        if (live && co < ly.cout) {
            if (ly.kind == L_CONV3)        // [cout][cin][3][3]
                v = theta[ly.w_off + ((int64_t)co * ly.cin + ci) * 9 + tap];
            else if (ly.kind == L_CONVT2)  // [cin][cout][2][2]
                v = theta[ly.w_off + ((int64_t)ci * ly.cout + co) * 4 + tap];
            else if (ly.kind == L_DOWN8)   // [cout][cin][8][8]
                v = theta[ly.w_off + ((int64_t)co * ly.cin + ci) * 64 + tap];
            else if (ly.kind == L_UP8)     // [cin][cout][8][8]
                v = theta[ly.w_off + ((int64_t)ci * ly.cout + co) * 64 + tap];
            else                           // [cout][cin][1][1]
                v = theta[ly.w_off + (int64_t)co * ly.cin + ci];
        }
        wb[ly.pk_off + idx] = f2bf(v);
        wf[ly.pk_off + idx] = v;
        wd[ly.pk_off + idx] = (double)v;
        if (ly.kind != L_CONV1) {
            // data-gradient pack [tap][cin_p][cout_p]: flipped taps for the 3x3 layers; for the 8x8
            // layers the same taps, which makes each one's data gradient the opposite 8x8 form
            const int tt = ly.kind == L_CONV3 ? 8 - tap : tap;
            const int64_t j = ((int64_t)tt * ly.cin_p + cis) * ly.cout_p + co;
            tb[ly.pk_off + j] = f2bf(v);
            tf[ly.pk_off + j] = v;
            td[ly.pk_off + j] = (double)v;
        }
    }
    if (idx < ly.cout_p) {
        const float b = idx < ly.cout ? theta[ly.b_off + idx] : 0.0f;
        bf[ly.bias_off + idx] = b;
        bd[ly.bias_off + idx] = (double)b;
    }
    if (idx == 0 && ly.a_off >= 0) {   // PReLU slope after the bias
        bf[ly.bias_off + ly.cout_p] = theta[ly.a_off];
        bd[ly.bias_off + ly.cout_p] = (double)theta[ly.a_off];
    }
}

static int repack_all(no_net* net, const float* theta, hipStream_t s) {
    hipLaunchKernelGGL(k_repack, dim3((unsigned)net->repack_blocks), dim3(256), 0, s, theta, net->layers_dev,
                       net->repack_start, (int)net->layers.size(), net->w_bf, net->w_f32, net->w_f64, net->b_f32,
                       net->b_f64, net->wt_bf, net->wt_f32, net->wt_f64);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int net_level_count(const no_net* net) { return net->a.levels; }

void net_padded_dims(const no_net* net, const hz_problem* p, int* Hp, int* Wp) {
    // UNET3: levels - 1 halvings; PAPER8: levels halvings
    const int m = 1 << (net->a.kind == NO_ARCH_PAPER8 ? net->a.levels : net->a.levels - 1);
    *Hp = (p->nyt + m - 1) / m * m;
    *Wp = (p->nxt + m - 1) / m * m;
}

// ------------------------------------------------------------------ pack / head

// s = ||v|| / sqrt(n) from norm partials; sc[0] = s, sc[1] = 1 / s (0 when s = 0).
__global__ void k_scale_factor(const double2* part, int nblk, int64_t n, double* sc, const int* skip) {
    if (skip && *skip) return;
    double a = 0;
    for (int q = threadIdx.x; q < nblk; q += 64) a += part[q].x;
    a = wave_sum(a);
    if (threadIdx.x == 0) {
        const double s = sqrt(a / (double)n);
        sc[0] = s;
        sc[1] = s > 0 ? 1.0 / s : 0.0;
    }
}

// z = s (out_0 + i out_1), out_k = sum_c D0[c] Wh[k][c] + bh[k], on the grid only.
template <class P, typename C>
__global__ void k_head(const typename P::T* __restrict__ D, int cin_p, const typename P::T* __restrict__ wh,
                       const typename P::Acc* __restrict__ bh, const double* __restrict__ sc, int nxt, int nyt,
                       int Wp, C* __restrict__ z, const int* __restrict__ skip, double fixed_s) {
    using Acc = typename P::Acc;
    if (skip && *skip) return;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nxt * nyt) return;
    const int yy = (int)(idx / nxt), xx = (int)(idx % nxt);
    using T = typename P::T;
    const T* d = D + ((int64_t)yy * Wp + xx) * cin_p;
    Acc o0 = bh[0], o1 = bh[1];
    // the pixel's channels in 16-byte loads (cin_p is a multiple of 8); same order of sums
    constexpr int V = 16 / (int)sizeof(T);
    for (int c = 0; c < cin_p; c += V) {
        const uint4 raw = *(const uint4*)(d + c);
        const T* e = (const T*)&raw;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const Acc dv = P::val(e[j]);
            o0 += dv * P::val(wh[c + j]);
            o1 += dv * P::val(wh[cin_p + c + j]);
        }
    }
    const double s = fixed_s > 0 ? fixed_s : sc[0];
    z[idx] = from_d2<C>(double2{s * (double)o0, s * (double)o1});
}

template <class P>
static int precond_impl(const no_net* net, const hz_problem* p, bool c128, const void* v, void* z, void* ws,
                        size_t ws_bytes, const int* skip, hipStream_t s, bool unit_norm,
                        const double* vscale, const NormParts* nparts) {
    using T = typename P::T;
    if ((vscale && !unit_norm) || (nparts && (unit_norm || vscale))) {
        set_error("no_precond_apply: in-place scaling needs a unit-norm result, a given scale neither");
        return HZ_ERR_ARG;
    }
    int Hp, Wp;
    net_padded_dims(net, p, &Hp, &Wp);
    FwdBufs b = fwd_layout<P>(net, Hp, Wp, 1, ws, ws_bytes);
    if (b.total > ws_bytes) {
        set_error("no_precond_apply: workspace too small");
        return HZ_ERR_WORKSPACE;
    }
    b.fuse_up = net->fuse_up;
    const int64_t n = p->n;
    Split sp = krylov_split(n);
    // s = ||v|| / sqrt(n); a unit-norm Krylov vector has s = 1 / sqrt(n) without a reduction
    const double fixed_s = unit_norm ? 1.0 / sqrt((double)n) : 0.0;
    double* scp = nparts ? nparts->sc : b.sc;   // [s, 1/s]
    if (!unit_norm && !nparts) {
        HZ_TRY(launch_norm_partials(c128, v, n, sp, b.part, 1, 0, skip, s));
        hipLaunchKernelGGL(k_scale_factor, dim3(1), dim3(64), 0, s, b.part, sp.nblk, n, b.sc, skip);
        HZ_LAUNCH_CHECK();
    }
    const unsigned gp = (unsigned)(((int64_t)Hp * Wp + 255) / 256);
    if (c128)
        hipLaunchKernelGGL((k_pack<P, double2>), dim3(gp), dim3(256), 0, s, (const double2*)v, scp, p->cnd, p->sigx,
                           p->sigy, p->nxt, p->nyt, Hp, Wp, net->a.in_ch, (T*)b.X, skip, fixed_s, vscale,
                           vscale ? (double2*)v : nullptr, nparts ? nparts->part : nullptr, nparts ? nparts->count : 0,
                           nparts ? nparts->ldp : 0);
    else
        hipLaunchKernelGGL((k_pack<P, float2>), dim3(gp), dim3(256), 0, s, (const float2*)v, scp, p->cnd, p->sigx,
                           p->sigy, p->nxt, p->nyt, Hp, Wp, net->a.in_ch, (T*)b.X, skip, fixed_s, vscale,
                           vscale ? (float2*)v : nullptr, nparts ? nparts->part : nullptr, nparts ? nparts->count : 0,
                           nparts ? nparts->ldp : 0);
    HZ_LAUNCH_CHECK();
    const Layer& lh = net->layers.back();
    if (net->a.kind == NO_ARCH_PAPER8) {
        HZ_TRY(paper8_body<P>(net, b, Hp, Wp, 1, skip, s));
        const unsigned gh = (unsigned)((n + 255) / 256);
        if (c128)
            hipLaunchKernelGGL((k_head<P, double2>), dim3(gh), dim3(256), 0, s, (const T*)b.U[0], lh.cin_p,
                               packed_w<P>(net, lh), packed_b<P>(net, lh), scp, p->nxt, p->nyt, Wp, (double2*)z, skip,
                               fixed_s);
        else
            hipLaunchKernelGGL((k_head<P, float2>), dim3(gh), dim3(256), 0, s, (const T*)b.U[0], lh.cin_p,
                               packed_w<P>(net, lh), packed_b<P>(net, lh), scp, p->nxt, p->nyt, Wp, (float2*)z, skip,
                               fixed_s);
        HZ_LAUNCH_CHECK();
        return HZ_OK;
    }
    if (lh.cin_p == 16 || lh.cin_p == 32 || lh.cin_p == 64) {
        // the head runs in the epilogue of the last 3x3 layer
        Conv3Out hd;
        hd.head_w = packed_w<P>(net, lh);
        hd.head_b = packed_b<P>(net, lh);
        hd.head_z = z;
        hd.head_c128 = c128 ? 1 : 0;
        hd.head_nxt = p->nxt;
        hd.head_nyt = p->nyt;
        hd.head_sc = scp;
        hd.head_fixed_s = fixed_s;
        return unet_body<P>(net, b, Hp, Wp, 1, skip, s, &hd);
    }
    HZ_TRY(unet_body<P>(net, b, Hp, Wp, 1, skip, s));
    const T* D0 = net->a.levels > 1 ? (const T*)b.D[0] : (const T*)b.E[0];
    const unsigned gh = (unsigned)((n + 255) / 256);
    if (c128)
        hipLaunchKernelGGL((k_head<P, double2>), dim3(gh), dim3(256), 0, s, D0, lh.cin_p, packed_w<P>(net, lh),
                           packed_b<P>(net, lh), scp, p->nxt, p->nyt, Wp, (double2*)z, skip, fixed_s);
    else
        hipLaunchKernelGGL((k_head<P, float2>), dim3(gh), dim3(256), 0, s, D0, lh.cin_p, packed_w<P>(net, lh),
                           packed_b<P>(net, lh), scp, p->nxt, p->nyt, Wp, (float2*)z, skip, fixed_s);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

ConvCfg net_cfg(const no_net* net, int layer, int H, int W, int batch, no_prec prec) {
    no_net* mnet = const_cast<no_net*>(net);
    std::lock_guard<std::mutex> g(mnet->tune_mu);
    auto it = mnet->tuned.find({layer, H, W, batch, (int)prec});
    return it == mnet->tuned.end() ? ConvCfg() : it->second;
}

constexpr int FUSED_KEY = 16;   // offset of the precision field in the keys of fused-form variants

ConvCfg net_cfg_up(const no_net* net, int layer, int H, int W, int batch, no_prec prec) {
    return net_cfg(net, layer, H, W, batch, (no_prec)((int)prec + FUSED_KEY));
}

// Holds the stream for `ticks` of the constant-rate wall clock (always returns), so that the
// launches queued behind it meanwhile run back to back: the autotuner then times the GPU, not the
// host's launch rate.
__global__ void k_hold(int64_t ticks) {
    const int64_t t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(8);
}

// Time the variants of every 3x3 layer on the forward buffers and keep the fastest. The
// candidates (channel tile, rows per wavefront) all accumulate every output in the same order,
// so the choice changes speed only, never a result bit; split-K (a different summation order)
// is not a candidate, which keeps solves reproducible whatever the timings were.
template <class P>
static int autotune_impl(const no_net* net, int Hp, int Wp, int batch, const FwdBufs& b, hipStream_t s) {
    using T = typename P::T;
    using Acc = typename P::Acc;
    no_net* mnet = const_cast<no_net*>(net);
    const int lv = net->a.levels;
    const std::vector<Layer>& Ls = net->layers;
    hipEvent_t e0, e1;
    HZ_HIP(hipEventCreate(&e0));
    HZ_HIP(hipEventCreate(&e1));
    int rc = HZ_OK;
    // 0.5 ms hold before each timed batch (the wall clock rate is reported in kHz)
    int dev = 0, wrate = 0;
    HZ_HIP(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&wrate, hipDeviceAttributeWallClockRate, dev) != hipSuccess || wrate <= 0) wrate = 100000;
    const int64_t hold_ticks = (int64_t)wrate / 2;
    auto hold = [&]() {
        hipLaunchKernelGGL(k_hold, dim3(1), dim3(64), 0, s, hold_ticks);
        return hipGetLastError() == hipSuccess ? HZ_OK : HZ_ERR_HIP;
    };
    // up (fused form): x1 is unused and U = convT2(up) is computed inside the layer
    // best_out (optional): average time of the chosen variant, ms per launch
    auto tune_layer = [&](int li, const T* x0, int c0, const T* x1, int c1, T* y, T* pool, int H, int W,
                          const UpIn* up = nullptr, float* best_out = nullptr) -> int {
        const std::array<int, 5> key{li, H, W, batch, (int)prec_of<P>() + (up ? FUSED_KEY : 0)};
        {
            std::lock_guard<std::mutex> g(mnet->tune_mu);
            if (mnet->tuned.count(key) && !best_out) return HZ_OK;
        }
        const Layer& ly = Ls[li];
        ConvCfg best;
        float best_ms = 1e30f;
        const int chunks = (c0 + c1) / std::max(1, std::min(P::CK, c1 > 0 ? std::min(c0, c1) : c0 + c1));
        // candidates: (channel tile, rows per wavefront) with 1 / 2 / 4 chunks per LDS stage, and the
        // weight-stationary form with 2 ... 16 tiles per block where it applies
        std::vector<ConvCfg> cands;
        for (int tn : {16, 32, 64}) {
            if (ly.cout_p % tn) continue;
            for (int rpw : {2, 4}) {
                for (int ns : {1, 2, 4}) {
                    // chunks per LDS stage: only where there are that many chunks (the plain form)
                    if (ns > 1 && (up || ns > chunks || !conv3_stages_ok<P>(tn, rpw, ns))) continue;
                    ConvCfg cfg{tn, rpw, 1};
                    cfg.ns = ns;
                    cands.push_back(cfg);
                }
                if (!up && conv3_ws_ok<P>(tn, rpw, c0, c1, ly.cout_p))
                    for (const auto& tp : {std::array<int, 2>{4, 2}, {8, 3}, {16, 3}, {16, 4}, {32, 4}}) {
                        // (tiles per block, tiles of loads in flight; 4 only with at most 2 chunks;
                        // 16-row tiles with 2)
                        if ((tp[1] == 4 && c0 + c1 > 2 * P::CK) || (rpw == 4 && tp[1] > 2)) continue;
                        ConvCfg cfg{tn, rpw, 1};
                        cfg.tpb = tp[0];
                        cfg.ns = tp[1];
                        cands.push_back(cfg);
                    }
            }
        }
        for (const ConvCfg& cfg : cands) {
            auto run = [&]() {
                if (up)
                    return launch_conv3_up<P>(x0, c0, *up, c1, packed_w<P>(net, ly), packed_b<P>(net, ly),
                                              y, ly.cout_p, H, W, batch, nullptr, s, cfg);
                return launch_conv3<P>(x0, c0, x1, c1, packed_w<P>(net, ly), packed_b<P>(net, ly), y,
                                       ly.cout_p, pool, H, W, batch, true, nullptr, s, Conv3Out(), cfg,
                                       (Acc*)b.splitbuf);
            };
            HZ_TRY(run());
            HZ_TRY(hold());
            HZ_HIP(hipEventRecord(e0, s));
            for (int r = 0; r < 10; ++r) HZ_TRY(run());
            HZ_HIP(hipEventRecord(e1, s));
            HZ_HIP(hipEventSynchronize(e1));
            float ms = 0;
            HZ_HIP(hipEventElapsedTime(&ms, e0, e1));
            // a later candidate replaces the current best only when clearly faster (3 %),
            // so that timing noise does not flip the choice between near-equal variants
            if (ms < 0.97f * best_ms) {
                best_ms = ms;
                best = cfg;
            }
        }
        if (best_out) *best_out = best_ms / 10;
        std::lock_guard<std::mutex> g(mnet->tune_mu);
        if (!mnet->tuned.count(key)) {
            mnet->tuned[key] = best;
            mnet->tune_gen.fetch_add(1);
        }
        return HZ_OK;
    };
    // average time of the stand-alone transposed convolution, ms per launch
    auto time_convT2 = [&](const Layer& lu, const T* x, T* y, int H, int W, float* ms_out) -> int {
        auto run = [&]() {
            return launch_convT2<P>(x, lu.cin_p, packed_w<P>(net, lu), packed_b<P>(net, lu), y, lu.cout_p, H, W,
                                    batch, nullptr, s);
        };
        HZ_TRY(run());
        HZ_TRY(hold());
        HZ_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 10; ++r) HZ_TRY(run());
        HZ_HIP(hipEventRecord(e1, s));
        HZ_HIP(hipEventSynchronize(e1));
        float ms = 0;
        HZ_HIP(hipEventElapsedTime(&ms, e0, e1));
        *ms_out = ms / 10;
        return HZ_OK;
    };
    int li = 0;
    for (int l = 0; l < lv && rc == HZ_OK; ++l) {
        const int H = Hp >> l, W = Wp >> l;
        const Layer& la = Ls[li];
        const T* in = l == 0 ? (const T*)b.X : (const T*)b.P[l];
        rc = tune_layer(li, in, la.cin_p, nullptr, 0, (T*)b.T1[l], nullptr, H, W);
        if (rc == HZ_OK)
            rc = tune_layer(li + 1, (const T*)b.T1[l], Ls[li + 1].cin_p, nullptr, 0, (T*)b.E[l],
                            l + 1 < lv ? (T*)b.P[l + 1] : nullptr, H, W);
        li += 2;
    }
    for (int l = lv - 2; l >= 0 && rc == HZ_OK; --l) {
        const int H = Hp >> l, W = Wp >> l;
        const Layer& lu = Ls[li];
        const int ce = lu.cout_p;
        const std::array<int, 5> ukey{li + 1, H, W, batch, (int)prec_of<P>() + FUSED_KEY};
        bool have_u;
        {
            std::lock_guard<std::mutex> g(mnet->tune_mu);
            have_u = mnet->tuned.count(ukey) > 0;
        }
        if (b.fuse_up && conv3_up_ok<P>(ce, ce, lu.cin_p, H, W) && !have_u) {
            // the fused form against the two separate layers (the same result bits): keep the
            // faster, by a clear margin for the fused form
            const T* dn = (const T*)(l + 1 == lv - 1 ? b.E[l + 1] : b.D[l + 1]);
            UpIn up;
            up.d = dn;
            up.cd = lu.cin_p;
            up.wt = packed_w<P>(net, lu);
            up.bt = packed_b<P>(net, lu);
            float t_fused = 0, t_conv = 0, t_up = 0;
            rc = tune_layer(li + 1, (const T*)b.E[l], ce, nullptr, ce, (T*)b.T1d[l], nullptr, H, W, &up, &t_fused);
            if (rc == HZ_OK)
                rc = tune_layer(li + 1, (const T*)b.E[l], ce, (const T*)b.U[l], ce, (T*)b.T1d[l], nullptr, H, W,
                                nullptr, &t_conv);
            if (rc == HZ_OK) rc = time_convT2(lu, dn, (T*)b.U[l], H / 2, W / 2, &t_up);
            if (rc == HZ_OK) {
                std::lock_guard<std::mutex> g(mnet->tune_mu);
                mnet->tuned[ukey].fuse = t_fused < 0.97f * (t_conv + t_up) ? 1 : 0;
                mnet->tune_gen.fetch_add(1);
            }
        } else {
            rc = tune_layer(li + 1, (const T*)b.E[l], ce, (const T*)b.U[l], ce, (T*)b.T1d[l], nullptr, H, W);
        }
        if (rc == HZ_OK)
            rc = tune_layer(li + 2, (const T*)b.T1d[l], Ls[li + 2].cin_p, nullptr, 0, (T*)b.D[l], nullptr, H, W);
        li += 3;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int net_autotune(const no_net* net, const hz_problem* p, no_prec prec, void* ws, size_t ws_bytes, hipStream_t s) {
    if (net->a.kind == NO_ARCH_PAPER8) return HZ_OK;   // one launch form per layer: nothing to tune
    int Hp, Wp;
    net_padded_dims(net, p, &Hp, &Wp);
    switch (prec) {
        case NO_BF16: {
            FwdBufs b = fwd_layout<PolBF16>(net, Hp, Wp, 1, ws, ws_bytes);
            if (b.total > ws_bytes) break;
            b.fuse_up = net->fuse_up;
            return autotune_impl<PolBF16>(net, Hp, Wp, 1, b, s);
        }
        case NO_FP32: {
            FwdBufs b = fwd_layout<PolF32>(net, Hp, Wp, 1, ws, ws_bytes);
            if (b.total > ws_bytes) break;
            b.fuse_up = net->fuse_up;
            return autotune_impl<PolF32>(net, Hp, Wp, 1, b, s);
        }
        case NO_FP64: {
            FwdBufs b = fwd_layout<PolF64>(net, Hp, Wp, 1, ws, ws_bytes);
            if (b.total > ws_bytes) break;
            b.fuse_up = net->fuse_up;
            return autotune_impl<PolF64>(net, Hp, Wp, 1, b, s);
        }
    }
    set_error("autotune: workspace too small or bad precision");
    return HZ_ERR_WORKSPACE;
}

int net_autotune_bufs(const no_net* net, int Hp, int Wp, int batch, const FwdBufs& b, no_prec prec, hipStream_t s) {
    if (net->a.kind == NO_ARCH_PAPER8) return HZ_OK;
    switch (prec) {
        case NO_BF16: return autotune_impl<PolBF16>(net, Hp, Wp, batch, b, s);
        case NO_FP32: return autotune_impl<PolF32>(net, Hp, Wp, batch, b, s);
        case NO_FP64: return autotune_impl<PolF64>(net, Hp, Wp, batch, b, s);
    }
    set_error("autotune: bad precision");
    return HZ_ERR_ARG;
}

size_t net_fwd_ws_bytes(const no_net* net, int Hp, int Wp, int batch, no_prec prec) {
    switch (prec) {
        case NO_BF16: return fwd_layout<PolBF16>(net, Hp, Wp, batch, nullptr, 0).total;
        case NO_FP32: return fwd_layout<PolF32>(net, Hp, Wp, batch, nullptr, 0).total;
        default: return fwd_layout<PolF64>(net, Hp, Wp, batch, nullptr, 0).total;
    }
}

int net_precond(const no_net* net, const hz_problem* p, no_prec prec, bool c128, const void* v, void* z, void* ws,
                size_t ws_bytes, const int* skip, hipStream_t s, bool unit_norm, const double* vscale,
                const NormParts* nparts) {
    switch (prec) {
        case NO_BF16:
            return precond_impl<PolBF16>(net, p, c128, v, z, ws, ws_bytes, skip, s, unit_norm, vscale, nparts);
        case NO_FP32:
            return precond_impl<PolF32>(net, p, c128, v, z, ws, ws_bytes, skip, s, unit_norm, vscale, nparts);
        case NO_FP64:
            return precond_impl<PolF64>(net, p, c128, v, z, ws, ws_bytes, skip, s, unit_norm, vscale, nparts);
    }
    set_error("no_precond_apply: bad precision");
    return HZ_ERR_ARG;
}

}  // namespace hz

using namespace hz;

extern "C" int64_t no_param_count(const no_arch* a) {
    std::vector<Layer> L;
    int64_t np, pk, nb;
    if (!build_layers(a, L, np, pk, nb)) return -1;
    return np;
}

extern "C" int no_net_create(const no_arch* a, const float* theta, void* stream, no_net** out) {
    clear_error();
    HZ_CHECK_ARG(a && theta && out, "no_net_create: NULL argument");
    no_net* net = new no_net();
    net->uid = next_handle_uid();
    if (!build_layers(a, net->layers, net->nparam, net->pk_total, net->bias_total)) {
        delete net;
        set_error("no_net_create: UNET3 needs levels 1..6 and base a multiple of 8, PAPER8 depth 1..5 and 32 "
                  "channels; in_ch 2 or 5");
        return HZ_ERR_ARG;
    }
    net->a = *a;
    const size_t nl = net->layers.size();
    const size_t bytes = 2 * net->pk_total * (2 + 4 + 8) + net->bias_total * (4 + 8) + nl * sizeof(Layer) +
                         (nl + 1) * sizeof(int64_t) + 10 * 256;
    if (hipMalloc(&net->block, bytes) != hipSuccess) {
        delete net;
        set_error("no_net_create: hipMalloc failed");
        return HZ_ERR_HIP;
    }
    Carver c(net->block, bytes);
    net->w_bf = c.take<bf16_t>(net->pk_total);
    net->w_f32 = c.take<float>(net->pk_total);
    net->w_f64 = c.take<double>(net->pk_total);
    net->b_f32 = c.take<float>(net->bias_total);
    net->b_f64 = c.take<double>(net->bias_total);
    net->wt_bf = c.take<bf16_t>(net->pk_total);
    net->wt_f32 = c.take<float>(net->pk_total);
    net->wt_f64 = c.take<double>(net->pk_total);
    net->layers_dev = c.take<Layer>(nl);
    net->repack_start = c.take<int64_t>(nl + 1);
    std::vector<int64_t> start(nl + 1, 0);
    for (size_t l = 0; l < nl; ++l) {
        const Layer& ly = net->layers[l];
        const int64_t n = std::max<int64_t>(ly.pk_len, ly.cout_p);
        start[l + 1] = start[l] + (n + 255) / 256;
    }
    net->repack_blocks = start[nl];
    hipStream_t s = (hipStream_t)stream;
    int rc = HZ_OK;
    if (hipMemcpy(net->layers_dev, net->layers.data(), nl * sizeof(Layer), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->repack_start, start.data(), (nl + 1) * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("no_net_create: copying the layer table failed");
        rc = HZ_ERR_HIP;
    }
    if (rc == HZ_OK) rc = repack_all(net, theta, s);
    if (rc == HZ_OK && hipStreamSynchronize(s) != hipSuccess) rc = HZ_ERR_HIP;
    if (rc != HZ_OK) {
        (void)hipFree(net->block);
        delete net;
        return rc;
    }
    *out = net;
    return HZ_OK;
}

extern "C" int no_net_set_weights(no_net* net, const float* theta, void* stream) {
    clear_error();
    HZ_CHECK_ARG(net && theta, "no_net_set_weights: NULL argument");
    return repack_all(net, theta, (hipStream_t)stream);
}

extern "C" int no_net_destroy(no_net* net) {
    clear_error();
    if (!net) return HZ_OK;
    fgmres_graph_cache_evict(net->uid);
    HZ_HIP(hipFree(net->block));
    delete net;
    return HZ_OK;
}

extern "C" size_t no_workspace_size(const no_net* net, const hz_problem* p, no_prec prec) {
    clear_error();
    if (!net || !p) return 0;
    int Hp, Wp;
    net_padded_dims(net, p, &Hp, &Wp);
    return net_fwd_ws_bytes(net, Hp, Wp, 1, prec);
}

extern "C" int no_precond_apply(const no_net* net, const hz_problem* p, no_prec prec, hz_dtype dtype, const void* v,
                                void* z, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    HZ_CHECK_ARG(net && p && v && z && ws, "no_precond_apply: NULL argument");
    HZ_CHECK_ARG(dtype == HZ_C64 || dtype == HZ_C128, "no_precond_apply: bad dtype");
    HZ_CHECK_ARG(v != z, "no_precond_apply: v and z must not overlap");
    return net_precond(net, p, prec, dtype == HZ_C128, v, z, ws, ws_bytes, nullptr, (hipStream_t)stream);
}

// ------------------------------------------------------------------ allocation-free forward pass

// Scratch memory of no_precond_apply_noalloc: one copy per GPU, held until the process ends. Host
// code never passes the array's name to a kernel (on the host it is only a stand-in symbol); the
// device address comes from hipGetSymbolAddress, once per device, and is kept in scratch_dev.
static __device__ __align__(256) unsigned char scratch[NO_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_dev[SCRATCH_MAX_DEVICES] = {};

// The current device's copy of `scratch` (looked up on the first call on that device).
int scratch_for_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_MAX_DEVICES) {
        set_error("no_precond_apply_noalloc: no usable current device");
        return HZ_ERR_HIP;
    }
    std::lock_guard<std::mutex> g(scratch_mu);
    if (!scratch_dev[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            set_error("no_precond_apply_noalloc: hipGetSymbolAddress of the scratch array failed");
            return HZ_ERR_HIP;
        }
        scratch_dev[dev] = ptr;
    }
    *out = scratch_dev[dev];
    return HZ_OK;
}
}  // namespace

extern "C" int no_precond_apply_noalloc(const no_net* net, const hz_problem* p, no_prec prec, hz_dtype dtype,
                                        const void* v, void* z, void* stream) {
    clear_error();
    HZ_CHECK_ARG(net && p && v && z, "no_precond_apply_noalloc: NULL argument");
    HZ_CHECK_ARG(dtype == HZ_C64 || dtype == HZ_C128, "no_precond_apply_noalloc: bad dtype");
    HZ_CHECK_ARG(prec == NO_BF16 || prec == NO_FP32 || prec == NO_FP64, "no_precond_apply_noalloc: bad precision");
    HZ_CHECK_ARG(v != z, "no_precond_apply_noalloc: v and z must not overlap");
    int Hp, Wp;
    net_padded_dims(net, p, &Hp, &Wp);
    const size_t need = net_fwd_ws_bytes(net, Hp, Wp, 1, prec);
    if (need > NO_NOALLOC_SCRATCH_BYTES) {
        set_error("no_precond_apply_noalloc: this grid and precision need " + std::to_string(need) +
                  " bytes of scratch, more than the fixed " + std::to_string((size_t)NO_NOALLOC_SCRATCH_BYTES) +
                  " (use no_precond_apply with a caller workspace)");
        return HZ_ERR_WORKSPACE;
    }
    void* ws = nullptr;
    HZ_TRY(scratch_for_current_device(&ws));
    return net_precond(net, p, prec, dtype == HZ_C128, v, z, ws, NO_NOALLOC_SCRATCH_BYTES, nullptr,
                       (hipStream_t)stream);
}

extern "C" int no_layer_info(const no_net* net, int layer, int32_t* kind, int32_t* cin_p, int32_t* cout_p,
                             int32_t* cat_cp) {
    clear_error();
    HZ_CHECK_ARG(net && layer >= 0 && layer < (int)net->layers.size(), "no_layer_info: bad layer");
    const Layer& ly = net->layers[layer];
    if (kind) *kind = ly.kind;
    if (cin_p) *cin_p = ly.cin_p;
    if (cout_p) *cout_p = ly.cout_p;
    if (cat_cp) *cat_cp = ly.cat_cp;
    return HZ_OK;
}

namespace hz {
template <class P>
static int layer_impl(const no_net* net, int layer, int batch, int H, int W, const void* x0, const void* x1,
                      void* y, void* pool, void* ws, size_t ws_bytes, hipStream_t s) {
    using T = typename P::T;
    const Layer& ly = net->layers[layer];
    if (ly.kind == L_DOWN8 || ly.kind == L_UP8)   // H, W: the input's size
        return launch_conv8<P>(ly.kind == L_UP8, (const T*)x0, (const T*)x1, ly.cin_p, ly.cat_cp,
                               packed_w<P>(net, ly), packed_b<P>(net, ly), (T*)y, ly.cout_p, H, W, batch, nullptr, s);
    if (ly.kind == L_CONV3) {
        const int c1 = ly.cat_cp ? ly.cin_p - ly.cat_cp : 0;
        const int c0 = ly.cin_p - c1;
        ConvCfg cfg = net_cfg(net, layer, H, W, batch, prec_of<P>());
        const size_t need = (size_t)cfg.ksplit * batch * H * W * ly.cout_p * sizeof(typename P::Acc);
        if (!ws || ws_bytes < need) cfg.ksplit = 1;
        return launch_conv3<P>((const T*)x0, c0, (const T*)x1, c1, packed_w<P>(net, ly), packed_b<P>(net, ly),
                               (T*)y, ly.cout_p, (T*)pool, H, W, batch, true, nullptr, s, Conv3Out(), cfg,
                               (typename P::Acc*)ws);
    }
    return launch_convT2<P>((const T*)x0, ly.cin_p, packed_w<P>(net, ly), packed_b<P>(net, ly), (T*)y, ly.cout_p,
                            H, W, batch, nullptr, s);
}
}  // namespace hz

extern "C" int no_layer_forward(const no_net* net, int layer, no_prec prec, int batch, int H, int W,
                                const void* x0, const void* x1, void* y, void* pool, void* ws, size_t ws_bytes,
                                void* stream) {
    clear_error();
    HZ_CHECK_ARG(net && layer >= 0 && layer < (int)net->layers.size() && x0 && y, "no_layer_forward: bad argument");
    const Layer& ly = net->layers[layer];
    HZ_CHECK_ARG(ly.kind != L_CONV1, "no_layer_forward: the head runs inside no_precond_apply only");
    HZ_CHECK_ARG(batch >= 1 && H >= 1 && W >= 1, "no_layer_forward: bad sizes");
    HZ_CHECK_ARG(!ly.cat_cp || x1, "no_layer_forward: concatenated input needs x1");
    HZ_CHECK_ARG(!pool || (ly.kind == L_CONV3 && H % 2 == 0 && W % 2 == 0), "no_layer_forward: bad pool output");
    hipStream_t s = (hipStream_t)stream;
    switch (prec) {
        case NO_BF16: return layer_impl<PolBF16>(net, layer, batch, H, W, x0, x1, y, pool, ws, ws_bytes, s);
        case NO_FP32: return layer_impl<PolF32>(net, layer, batch, H, W, x0, x1, y, pool, ws, ws_bytes, s);
        case NO_FP64: return layer_impl<PolF64>(net, layer, batch, H, W, x0, x1, y, pool, ws, ws_bytes, s);
    }
    set_error("no_layer_forward: bad precision");
    return HZ_ERR_ARG;
}

extern "C" int no_layer_variant(const no_net* net, int layer, no_prec prec, int batch, int H, int W, int32_t* tn,
                                int32_t* rows, int32_t* stages, int32_t* tiles) {
    clear_error();
    HZ_CHECK_ARG(net && tn && rows && stages && tiles, "no_layer_variant: NULL argument");
    HZ_CHECK_ARG(layer >= 0 && layer < (int)net->layers.size() && net->layers[layer].kind == L_CONV3,
                 "no_layer_variant: not a 3x3 layer");
    const ConvCfg c = net_cfg(net, layer, H, W, batch, prec);
    *tn = c.tn;
    *rows = 4 * (c.rpw == 4 ? 4 : 2);
    *stages = c.ns;
    *tiles = c.tpb > 1 ? c.tpb : 1;
    return HZ_OK;
}

extern "C" int no_set_layer_variant(const no_net* net, int layer, no_prec prec, int batch, int H, int W, int tn,
                                    int rows, int stages, int tiles) {
    clear_error();
    HZ_CHECK_ARG(net, "no_set_layer_variant: NULL network");
    HZ_CHECK_ARG(layer >= 0 && layer < (int)net->layers.size() && net->layers[layer].kind == L_CONV3,
                 "no_set_layer_variant: not a 3x3 layer");
    HZ_CHECK_ARG(prec == NO_BF16 || prec == NO_FP32 || prec == NO_FP64, "no_set_layer_variant: bad precision");
    HZ_CHECK_ARG((tn == 16 || tn == 32 || tn == 64) && net->layers[layer].cout_p % tn == 0 && (rows == 8 || rows == 16),
                 "no_set_layer_variant: tn must be 16, 32 or 64 and divide the output channels, rows 8 or 16");
    const int rpw = rows / 4;
    const Layer& ly = net->layers[layer];
    const int c0 = ly.cat_cp > 0 ? ly.cat_cp : ly.cin_p, c1 = ly.cat_cp > 0 ? ly.cin_p - ly.cat_cp : 0;
    if (tiles > 1) {
        HZ_CHECK_ARG(tiles <= 64 && prec == NO_BF16 && conv3_ws_ok<PolBF16>(tn, rpw, c0, c1, ly.cout_p) &&
                         stages >= 2 && stages <= (rpw == 4 ? 2 : c0 + c1 <= 2 * PolBF16::CK ? 4 : 3),
                     "no_set_layer_variant: tiles must be 1, or 2..64 for the weight-stationary BF16 form (at most "
                     "4 input chunks, LDS within 160 KB) with 2 or 3 tiles of loads in flight (4 with at most 2 "
                     "chunks)");
    } else {
        const bool st_ok = prec == NO_BF16 ? conv3_stages_ok<PolBF16>(tn, rpw, stages) : stages == 1;
        HZ_CHECK_ARG(st_ok && tiles == 1,
                     "no_set_layer_variant: stages must be 1, or 2 / 4 in BF16 where the stages fit in the LDS");
    }
    HZ_CHECK_ARG(batch >= 1 && H >= 1 && W >= 1, "no_set_layer_variant: bad size");
    no_net* mnet = const_cast<no_net*>(net);
    std::lock_guard<std::mutex> g(mnet->tune_mu);
    ConvCfg c{tn, rpw, 1};
    c.ns = stages;
    c.tpb = tiles > 1 ? tiles : 0;
    mnet->tuned[{layer, H, W, batch, (int)prec}] = c;
    mnet->tune_gen.fetch_add(1);
    return HZ_OK;
}

extern "C" int no_set_fused_upsampling(no_net* net, int mode) {
    clear_error();
    HZ_CHECK_ARG(net, "no_set_fused_upsampling: NULL network");
    HZ_CHECK_ARG(mode >= 0 && mode <= 2, "no_set_fused_upsampling: mode must be 0, 1 or 2");
    if (net->fuse_up != mode) net->tune_gen.fetch_add(1);
    net->fuse_up = mode;
    return HZ_OK;
}

extern "C" int no_autotune(const no_net* net, const hz_problem* p, no_prec prec, void* ws, size_t ws_bytes,
                           void* stream) {
    clear_error();
    HZ_CHECK_ARG(net && p && ws, "no_autotune: NULL argument");
    HZ_CHECK_ARG(prec == NO_BF16 || prec == NO_FP32 || prec == NO_FP64, "no_autotune: bad precision");
    return net_autotune(net, p, prec, ws, ws_bytes, (hipStream_t)stream);
}
