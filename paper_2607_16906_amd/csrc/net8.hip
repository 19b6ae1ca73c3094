// Layers of the paper's own U-Net (Section 3.1, Table 2): 8x8 convolutions with stride 2 and
// padding 3 (down: halves each side) and their transposed form (up: doubles each side), bias and
// PReLU (one slope per layer) in the epilogue, batch normalisation folded into the weights.
//
//   down: y[o][i][j] = b[o] + sum_{c,a,e} W[o][c][a][e] x[c][2i + a - 3][2j + e - 3]
//   up:   y[o][2i + a - 3][2j + e - 3] += W[c][o][a][e] x[c][i][j], then + b[o]
//
// Both are implicit GEMMs on the matrix cores with M = output channels, N = output pixels and
// K = taps x input channels. For the transposed form an output pixel of parity (py, px) receives
// exactly the 4 x 4 taps a = (py + 1) % 2 + 2 u, e = (px + 1) % 2 + 2 w (u, w = 0..3) from the
// input pixels (i + (py + 3 - a) / 2, j + (px + 3 - e) / 2); every wavefront therefore works on
// pixels of one parity class, which share their weights, and K = 16 x input channels.
//
// Activations are NHWC (channels padded to a multiple of 8, the first layer's input has 8); the
// packed weights are [tap = 8 a + e][cout_p][cin_p]; bias[cout_p] holds the PReLU slope. A
// wavefront owns 2 tiles of 16 pixels and all output channels (2 tiles of 16): each K step loads
// one B fragment per pixel tile straight from the (cache-resident) input and one A fragment per
// channel tile, and issues 4 matrix instructions.
#include "net.h"
#include "net_kernels.h"

namespace hz {

constexpr int C8_WAVES = 4;   // wavefronts per block
constexpr int C8_PX = 32;     // output pixels per wavefront

template <class P, bool UP>
__global__ __launch_bounds__(64 * C8_WAVES) void k_conv8(
    const typename P::T* __restrict__ x0, const typename P::T* __restrict__ x1, int cin_p, int cat_cp,
    const typename P::T* __restrict__ w, const typename P::Acc* __restrict__ bias, typename P::T* __restrict__ y,
    int Hin, int Win, int batch, int tiles, const int* __restrict__ skip) {
    using T = typename P::T;
    using Acc = typename P::Acc;
    using Frag = typename P::Frag;
    using AccV = typename P::AccV;
    constexpr int COUT = 32;
    constexpr int KSTEP = 4 * P::GW;
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63;
    const int64_t item = (int64_t)blockIdx.x * C8_WAVES + (threadIdx.x >> 6);
    constexpr int NCLS = UP ? 4 : 1;
    if (item >= (int64_t)batch * NCLS * tiles) return;   // whole wavefronts; no block barrier follows
    const int tile = (int)(item % tiles);
    const int bc = (int)(item / tiles);
    const int cls = bc % NCLS;
    const int b = bc / NCLS;
    const int py = cls >> 1, px = cls & 1;
    const int Ho = UP ? 2 * Hin : Hin / 2, Wo = UP ? 2 * Win : Win / 2;
    const int Hq = UP ? Hin : Ho, Wq = UP ? Win : Wo;   // pixels of one class
    const int col = lane & 15, g = lane >> 4;
    int qy[2], qx[2];
    bool qv[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int q = tile * C8_PX + t * 16 + col;
        qv[t] = q < Hq * Wq;
        qy[t] = qv[t] ? q / Wq : 0;
        qx[t] = qv[t] ? q % Wq : 0;
    }
    const int cs0 = cat_cp > 0 ? cat_cp : cin_p;   // channel stride of x0
    const int cs1 = cin_p - cat_cp;                // channel stride of x1 (concat only)
    const T* xb0 = x0 + (int64_t)b * Hin * Win * cs0;
    const T* xb1 = cat_cp > 0 ? x1 + (int64_t)b * Hin * Win * cs1 : nullptr;
    AccV acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[m][t][r] = 0;
    const int K = (UP ? 16 : 64) * cin_p;
    for (int k0 = 0; k0 < K; k0 += KSTEP) {
        const int k = k0 + g * P::GW;
        const int tap = k / cin_p, ci = k - tap * cin_p;
        int a, e, dy, dx;
        if (UP) {
            a = ((py + 1) & 1) + 2 * (tap >> 2);
            e = ((px + 1) & 1) + 2 * (tap & 3);
            dy = (py + 3 - a) >> 1;   // even numerator: exact
            dx = (px + 3 - e) >> 1;
        } else {
            a = tap >> 3;
            e = tap & 7;
            dy = a - 3;
            dx = e - 3;
        }
        const bool second = cat_cp > 0 && ci >= cat_cp;
        const T* src = second ? xb1 : xb0;
        const int cstr = second ? cs1 : cs0;
        const int cc = second ? ci - cat_cp : ci;
        Frag bf[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int iy = UP ? qy[t] + dy : 2 * qy[t] + dy;
            const int ix = UP ? qx[t] + dx : 2 * qx[t] + dx;
            const bool ok = qv[t] && iy >= 0 && iy < Hin && ix >= 0 && ix < Win;
            bf[t] = ok ? P::load(src + ((int64_t)iy * Win + ix) * cstr + cc) : P::zero();
        }
        const T* wt = w + ((int64_t)(a * 8 + e) * COUT + col) * cin_p + ci;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const Frag af = P::load(wt + (int64_t)m * 16 * cin_p);
#pragma unroll
            for (int t = 0; t < 2; ++t) acc[m][t] = P::mma(af, bf[t], acc[m][t]);
        }
    }
    const Acc slope = bias[COUT];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        if (!qv[t]) continue;
        const int oy = UP ? 2 * qy[t] + py : qy[t];
        const int ox = UP ? 2 * qx[t] + px : qx[t];
        T* dst = y + (((int64_t)b * Ho + oy) * Wo + ox) * COUT;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            Acc v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const Acc s = acc[m][t][r] + bias[m * 16 + P::row_of(g, r)];
                v[r] = s > 0 ? s : slope * s;
            }
            store_rows<P>(dst + m * 16 + P::row_of(g, 0), v);
        }
    }
}

template <class P>
int launch_conv8(bool up, const typename P::T* x0, const typename P::T* x1, int cin_p, int cat_cp,
                 const typename P::T* w, const typename P::Acc* bias, typename P::T* y, int cout_p, int Hin, int Win,
                 int batch, const int* skip, hipStream_t s) {
    // shapes the kernel assumes: 32 output channels, input channels in whole K steps (a step of
    // 4 GW values may span several taps when cin_p < 4 GW), even input sides for the down form
    if (cout_p != 32 || cin_p < P::GW || cin_p % P::GW || cin_p > 64 || ((up ? 16 : 64) * cin_p) % (4 * P::GW) ||
        (cat_cp > 0 && (!x1 || cat_cp % P::GW || cat_cp >= cin_p)) || Hin < 1 || Win < 1 || batch < 1 ||
        (!up && (Hin % 2 || Win % 2))) {
        set_error("conv8: unsupported layer shape");
        return HZ_ERR_ARG;
    }
    const int64_t px = up ? (int64_t)Hin * Win : (int64_t)(Hin / 2) * (Win / 2);
    const int tiles = (int)((px + C8_PX - 1) / C8_PX);
    const int64_t items = (int64_t)batch * (up ? 4 : 1) * tiles;
    const unsigned grid = (unsigned)((items + C8_WAVES - 1) / C8_WAVES);
    if (up)
        hipLaunchKernelGGL((k_conv8<P, true>), dim3(grid), dim3(64 * C8_WAVES), 0, s, x0, x1, cin_p, cat_cp, w, bias,
                           y, Hin, Win, batch, tiles, skip);
    else
        hipLaunchKernelGGL((k_conv8<P, false>), dim3(grid), dim3(64 * C8_WAVES), 0, s, x0, x1, cin_p, cat_cp, w,
                           bias, y, Hin, Win, batch, tiles, skip);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

template int launch_conv8<PolBF16>(bool, const bf16_t*, const bf16_t*, int, int, const bf16_t*, const float*, bf16_t*,
                                   int, int, int, int, const int*, hipStream_t);
template int launch_conv8<PolF32>(bool, const float*, const float*, int, int, const float*, const float*, float*, int,
                                  int, int, int, const int*, hipStream_t);
template int launch_conv8<PolF64>(bool, const double*, const double*, int, int, const double*, const double*, double*,
                                  int, int, int, int, const int*, hipStream_t);

}  // namespace hz
