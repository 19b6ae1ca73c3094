// Forward-pass plumbing shared by inference (net.hip) and training (train.hip).
#pragma once

#include <algorithm>
#include <vector>

#include "net.h"
#include "net_kernels.h"

namespace hz {

inline int round16(int c) { return (c + 15) / 16 * 16; }

// X[y][x][0..7] = [Re v / s, Im v / s, (c / c_ref, sigma_x, sigma_y), 0...] on the grid, 0 in the
// padding, for padded pixel idx; is = 1 / s. vscale: v <- vscale v first (rounded to the vector
// precision, stored back through vout). skipped: every input is loaded first and nothing is
// written (the caller's step-skip flag, whose load then overlaps these).
template <class P, typename C>
__device__ __forceinline__ void pack_pixel(const C* __restrict__ v, double is, const double* __restrict__ cnd,
                                           const double* __restrict__ sigx, const double* __restrict__ sigy, int nxt,
                                           int nyt, int Wp, int in_ch, typename P::T* __restrict__ X, int64_t idx,
                                           const double* __restrict__ vscale, C* vout, int skipped = 0) {
    using T = typename P::T;
    const int yy = (int)(idx / Wp), xx = (int)(idx % Wp);
    const bool on_grid = yy < nyt && xx < nxt;
    const int64_t g = (int64_t)yy * nxt + xx;
    C a{};
    double f = 1.0, cn = 0.0, sx = 0.0, sy = 0.0;
    if (on_grid) {
        a = v[g];
        if (vscale) f = *vscale;
        if (in_ch == 5) {
            cn = cnd[g];
            sx = sigx[xx];
            sy = sigy[yy];
        }
    }
    asm volatile("" ::: "memory");   // the loads stay above the test
    if (skipped) return;
    __attribute__((aligned(16))) T out[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) out[c] = P::cvt(0);
    if (on_grid) {
        if (vscale) {
            a = from_d2<C>(double2{a.x * f, a.y * f});
            vout[g] = a;
        }
        out[0] = P::cvt((typename P::Acc)((double)a.x * is));
        out[1] = P::cvt((typename P::Acc)((double)a.y * is));
        if (in_ch == 5) {
            out[2] = P::cvt((typename P::Acc)cn);
            out[3] = P::cvt((typename P::Acc)sx);
            out[4] = P::cvt((typename P::Acc)sy);
        }
    }
    T* dst = X + idx * 8;   // 8 channels per pixel: 16 B (BF16) or whole 16-byte vectors
    static_assert((8 * sizeof(T)) % 16 == 0, "pack: 8 channels must be whole 16-byte vectors");
#pragma unroll
    for (int c = 0; c < 8; c += 16 / (int)sizeof(T)) *(uint4*)(dst + c) = *(const uint4*)(out + c);
}

// One padded pixel per thread. fixed_s > 0: the caller knows ||v|| / sqrt(n) (a unit-norm Krylov
// vector) and sc is not read; otherwise s = 1 / sc[1].
template <class P, typename C>
//
// npart (with nnp, ldp): ||v||^2 is given as nnp partial sums npart[q * ldp].x (the caller's last
// pass over v wrote them); every block adds them in the same fixed order, and block 0 stores
// sc[0] = s, sc[1] = 1 / s for the later output scaling.
__global__ void k_pack(const C* __restrict__ v, double* __restrict__ sc, const double* __restrict__ cnd,
                       const double* __restrict__ sigx, const double* __restrict__ sigy, int nxt, int nyt, int Hp,
                       int Wp, int in_ch, typename P::T* __restrict__ X, const int* __restrict__ skip,
                       double fixed_s = 0.0, const double* __restrict__ vscale = nullptr, C* vout = nullptr,
                       const double2* __restrict__ npart = nullptr, int nnp = 0, int ldp = 0) {
    const int skipped = skip ? *skip : 0;   // tested after the pixel's loads (see pack_pixel)
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double is;
    if (npart) {
        if (skipped) return;   // uniform over the block
        __shared__ double red[4];
        double a = 0;
        for (int q = threadIdx.x; q < nnp; q += blockDim.x) a += npart[(int64_t)q * ldp].x;
        a = wave_sum(a);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
        __syncthreads();
        const double nv2 = red[0] + red[1] + red[2] + red[3];
        const double s = sqrt(nv2 / ((double)nxt * nyt));
        is = s > 0 ? 1.0 / s : 0.0;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc[0] = s;
            sc[1] = is;
        }
    } else {
        is = fixed_s > 0 ? 1.0 / fixed_s : sc[1];
    }
    if (idx >= (int64_t)Hp * Wp) return;
    pack_pixel<P, C>(v, is, cnd, sigx, sigy, nxt, nyt, Wp, in_ch, X, idx, vscale, vout, skipped);
}


// ------------------------------------------------------------------ forward

struct FwdBufs {
    void* X;
    std::vector<void*> E, T1, T1d, P, U, D;   // T1d: decoder temporaries (alias T1 for inference)
    double2* part;
    double* sc;
    void* splitbuf;      // split-K partial sums (accumulator type)
    size_t split_elems;
    size_t total;
    // inference: decoder levels may take the transposed convolution inside their first 3x3
    // convolution where that form applies (U is then not written): 0 never, 1 always, 2 where
    // the autotuner found it faster
    int fuse_up = 0;
};

// Autotune the 3x3 layers for `batch` samples on the forward buffers b (see no_autotune); layers
// already tuned at that size return at once. Synchronises the stream on the first call of a size.
int net_autotune_bufs(const no_net* net, int Hp, int Wp, int batch, const FwdBufs& b, no_prec prec, hipStream_t s);

template <class P>
inline FwdBufs fwd_layout(const no_net* net, int Hp, int Wp, int batch, void* base, size_t cap,
                          bool keep_all = false, bool recompute = false) {
    using T = typename P::T;
    FwdBufs b;
    Carver c(base, cap);
    const int lv = net->a.levels;
    b.X = c.take<T>((size_t)batch * Hp * Wp * 8);
    if (net->a.kind == NO_ARCH_PAPER8) {
        // E[l], l = 1..lv: encoder outputs at 1 / 2^l; U[l], l = 0..lv-1: decoder outputs at 1 / 2^l
        const int ch = net->a.base;
        b.E.assign(lv + 1, nullptr);
        b.U.assign(lv, nullptr);
        for (int l = 1; l <= lv; ++l) b.E[l] = c.take<T>((size_t)batch * (Hp >> l) * (Wp >> l) * ch);
        for (int l = 0; l < lv; ++l) b.U[l] = c.take<T>((size_t)batch * (Hp >> l) * (Wp >> l) * ch);
        b.part = c.take<double2>(1024);
        b.sc = c.take<double>(2);
        b.split_elems = 0;
        b.splitbuf = nullptr;
        b.total = c.off + 256;
        return b;
    }
    b.E.resize(lv);
    b.T1.resize(lv);
    b.T1d.resize(lv);
    b.P.resize(lv);
    b.U.resize(lv);
    b.D.resize(lv);
    // recompute (training with activation checkpointing): the first-convolution outputs (T1, T1d)
    // and the upsampled tensors (U) of every level share one scratch of the largest level's size
    // each; the backward pass recomputes them level by level
    T* t1s = nullptr;
    T* us = nullptr;
    if (recompute) {
        const size_t px0 = (size_t)batch * Hp * Wp;
        size_t mx = 0;
        for (int l = 0; l < lv; ++l) mx = std::max(mx, (px0 >> (2 * l)) * round16(net->a.base << l));
        t1s = c.take<T>(mx);
        us = c.take<T>(mx);
    }
    for (int l = 0; l < lv; ++l) {
        const size_t px = (size_t)batch * (Hp >> l) * (Wp >> l);
        const int cs = round16(net->a.base << l);
        b.E[l] = c.take<T>(px * cs);
        b.T1[l] = recompute ? t1s : c.take<T>(px * cs);
        b.T1d[l] = recompute ? t1s : (keep_all ? c.take<T>(px * cs) : b.T1[l]);
        b.P[l] = l > 0 ? c.take<T>(px * round16(net->a.base << (l - 1))) : nullptr;
        b.U[l] = l < lv - 1 ? (recompute ? us : c.take<T>(px * cs)) : nullptr;
        b.D[l] = l < lv - 1 ? c.take<T>(px * cs) : nullptr;
    }
    b.part = c.take<double2>(1024);
    b.sc = c.take<double>(2);
    // no split-K partials: the network's launches accumulate each output in one block (a split
    // would change the summation order with the launch variant)
    b.split_elems = 0;
    b.splitbuf = nullptr;
    b.total = c.off + 256;
    return b;
}

template <class P>
inline const typename P::T* packed_w(const no_net* net, const Layer& ly) {
    if constexpr (sizeof(typename P::T) == 2) return net->w_bf + ly.pk_off;
    else if constexpr (sizeof(typename P::T) == 4) return net->w_f32 + ly.pk_off;
    else return net->w_f64 + ly.pk_off;
}
// data-gradient packs: 3x3 layers [tap'][cin_p][cout_p] with tap' = 8 - tap, transposed
// convolutions [ab][cin_p][cout_p]
template <class P>
inline const typename P::T* packed_wt(const no_net* net, const Layer& ly) {
    if constexpr (sizeof(typename P::T) == 2) return net->wt_bf + ly.pk_off;
    else if constexpr (sizeof(typename P::T) == 4) return net->wt_f32 + ly.pk_off;
    else return net->wt_f64 + ly.pk_off;
}
template <class P>
inline const typename P::Acc* packed_b(const no_net* net, const Layer& ly) {
    if constexpr (sizeof(typename P::Acc) == 4) return net->b_f32 + ly.bias_off;
    else return net->b_f64 + ly.bias_off;
}

// Network body on a packed input X (batch samples), result D0 = decoder level-0 output.
template <class P>
constexpr no_prec prec_of() {
    return sizeof(typename P::T) == 2 ? NO_BF16 : (sizeof(typename P::T) == 4 ? NO_FP32 : NO_FP64);
}

// Body of the paper's own network (NO_ARCH_PAPER8) on a packed input X: encoder E[1..lv], decoder
// U[lv-1..0]; the 1x1 head reads U[0].
template <class P>
inline int paper8_body(const no_net* net, const FwdBufs& b, int Hp, int Wp, int batch, const int* skip,
                       hipStream_t s) {
    using T = typename P::T;
    const int lv = net->a.levels;
    const std::vector<Layer>& Ls = net->layers;
    int li = 0;
    const T* in = (const T*)b.X;
    for (int l = 1; l <= lv; ++l) {
        const Layer& ly = Ls[li++];
        HZ_TRY(launch_conv8<P>(false, in, nullptr, ly.cin_p, 0, packed_w<P>(net, ly), packed_b<P>(net, ly),
                               (T*)b.E[l], ly.cout_p, Hp >> (l - 1), Wp >> (l - 1), batch, skip, s));
        in = (const T*)b.E[l];
    }
    {
        const Layer& ly = Ls[li++];
        HZ_TRY(launch_conv8<P>(true, (const T*)b.E[lv], nullptr, ly.cin_p, 0, packed_w<P>(net, ly),
                               packed_b<P>(net, ly), (T*)b.U[lv - 1], ly.cout_p, Hp >> lv, Wp >> lv, batch, skip, s));
    }
    for (int l = lv - 2; l >= 0; --l) {
        const Layer& ly = Ls[li++];
        HZ_TRY(launch_conv8<P>(true, (const T*)b.E[l + 1], (const T*)b.U[l + 1], ly.cin_p, ly.cat_cp,
                               packed_w<P>(net, ly), packed_b<P>(net, ly), (T*)b.U[l], ly.cout_p, Hp >> (l + 1),
                               Wp >> (l + 1), batch, skip, s));
    }
    return HZ_OK;
}

template <class P>
inline int unet_body(const no_net* net, const FwdBufs& b, int Hp, int Wp, int batch, const int* skip, hipStream_t s,
                     const Conv3Out* head = nullptr) {
    using Acc = typename P::Acc;
    Acc* sb = (Acc*)b.splitbuf;
    using T = typename P::T;
    const int lv = net->a.levels;
    const std::vector<Layer>& Ls = net->layers;
    int li = 0;
    for (int l = 0; l < lv; ++l) {
        const int H = Hp >> l, W = Wp >> l;
        const Layer& la = Ls[li++];
        const Layer& lb = Ls[li++];
        const T* in = l == 0 ? (const T*)b.X : (const T*)b.P[l];
        HZ_TRY(launch_conv3<P>(in, la.cin_p, nullptr, 0, packed_w<P>(net, la), packed_b<P>(net, la), (T*)b.T1[l],
                               la.cout_p, nullptr, H, W, batch, true, skip, s, Conv3Out(),
                               net_cfg(net, li - 2, H, W, batch, prec_of<P>()), sb));
        T* pool = l + 1 < lv ? (T*)b.P[l + 1] : nullptr;
        const bool last = lv == 1 && head;   // a one-level net ends here
        HZ_TRY(launch_conv3<P>((const T*)b.T1[l], lb.cin_p, nullptr, 0, packed_w<P>(net, lb), packed_b<P>(net, lb),
                               (T*)b.E[l], lb.cout_p, pool, H, W, batch, true, skip, s, last ? *head : Conv3Out(),
                               net_cfg(net, li - 1, H, W, batch, prec_of<P>()), sb));
    }
    const T* Dn = (const T*)b.E[lv - 1];
    for (int l = lv - 2; l >= 0; --l) {
        const int H = Hp >> l, W = Wp >> l;
        const Layer& lu = Ls[li++];
        const Layer& la = Ls[li++];
        const Layer& lb = Ls[li++];
        const int ce = lu.cout_p;
        const ConvCfg ucfg = net_cfg_up(net, li - 2, H, W, batch, prec_of<P>());
        if (conv3_up_ok<P>(ce, ce, lu.cin_p, H, W) && (b.fuse_up == 1 || (b.fuse_up == 2 && ucfg.fuse))) {
            UpIn up;
            up.d = Dn;
            up.cd = lu.cin_p;
            up.wt = packed_w<P>(net, lu);
            up.bt = packed_b<P>(net, lu);
            HZ_TRY(launch_conv3_up<P>((const T*)b.E[l], ce, up, ce, packed_w<P>(net, la), packed_b<P>(net, la),
                                      (T*)b.T1d[l], la.cout_p, H, W, batch, skip, s, ucfg));
        } else {
            HZ_TRY(launch_convT2<P>(Dn, lu.cin_p, packed_w<P>(net, lu), packed_b<P>(net, lu), (T*)b.U[l],
                                    lu.cout_p, H / 2, W / 2, batch, skip, s));
            HZ_TRY(launch_conv3<P>((const T*)b.E[l], ce, (const T*)b.U[l], ce, packed_w<P>(net, la),
                                   packed_b<P>(net, la), (T*)b.T1d[l], la.cout_p, nullptr, H, W, batch, true, skip,
                                   s, Conv3Out(), net_cfg(net, li - 2, H, W, batch, prec_of<P>()), sb));
        }
        const bool last = l == 0 && head;
        HZ_TRY(launch_conv3<P>((const T*)b.T1d[l], lb.cin_p, nullptr, 0, packed_w<P>(net, lb), packed_b<P>(net, lb),
                               (T*)b.D[l], lb.cout_p, nullptr, H, W, batch, true, skip, s, last ? *head : Conv3Out(),
                               net_cfg(net, li - 1, H, W, batch, prec_of<P>()), sb));
        Dn = (const T*)b.D[l];
    }
    return HZ_OK;
}

}  // namespace hz
