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
// packed weights are [tap = 8 a + e][cout_p][cin_p]; bias[cout_p] holds the PReLU slope. An item
// is 2 tiles of 16 pixels and all output channels (2 tiles of 16): each K step loads one B
// fragment per pixel tile straight from the (cache-resident) input and one A fragment per channel
// tile, and issues 4 matrix instructions. Small layers split an item's K steps over several
// wavefronts so that the grid still fills the chip.
#include "net.h"
#include "net_kernels.h"

namespace hz {

constexpr int C8_PX = 32;     // output pixels per wavefront

// ks wavefronts of a block share one item (2 x 16 pixels, all 32 output channels) and split its K
// steps into ks consecutive ranges; the partial sums meet in LDS (dynamic, nw x 16 x 64
// accumulators) and the first wavefront of the group finishes the item. A block has nw = 4 or 8
// wavefronts and holds nw / ks items.
template <class P, bool UP>
__global__ __launch_bounds__(512) void k_conv8(
    const typename P::T* __restrict__ x0, const typename P::T* __restrict__ x1, int cin_p, int cat_cp,
    const typename P::T* __restrict__ w, const typename P::Acc* __restrict__ bias, typename P::T* __restrict__ y,
    int Hin, int Win, int batch, int tiles, int ks, const int* __restrict__ skip, typename P::T* __restrict__ ypre,
    int wcout) {
    using T = typename P::T;
    using Acc = typename P::Acc;
    using Frag = typename P::Frag;
    using AccV = typename P::AccV;
    constexpr int COUT = 32;
    constexpr int KSTEP = 4 * P::GW;
    extern __shared__ __align__(16) unsigned char c8_smem[];
    if (skip && *skip) return;   // uniform over the block
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int kw = wv % ks;
    const int64_t item = (int64_t)blockIdx.x * (nw / ks) + wv / ks;
    constexpr int NCLS = UP ? 4 : 1;
    const bool live = item < (int64_t)batch * NCLS * tiles;   // dead wavefronts still meet the barrier
    const int tile = live ? (int)(item % tiles) : 0;
    const int bc = live ? (int)(item / tiles) : 0;
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
        qv[t] = live && q < Hq * Wq;
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
    const int nsteps = (UP ? 16 : 64) * cin_p / KSTEP;
    const int per = nsteps / ks;
    const int s0 = kw * per;
    const int s1 = live ? (kw + 1) * per : s0;
    // fragments of K step st: B (input) per pixel tile, A (weights) per channel tile
    auto load_step = [&](int st, Frag (&bf)[2], Frag (&af)[2]) {
        const int k = st * KSTEP + g * P::GW;
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
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int iy = UP ? qy[t] + dy : 2 * qy[t] + dy;
            const int ix = UP ? qx[t] + dx : 2 * qx[t] + dx;
            const bool ok = qv[t] && iy >= 0 && iy < Hin && ix >= 0 && ix < Win;
            bf[t] = ok ? P::load(src + ((int64_t)iy * Win + ix) * cstr + cc) : P::zero();
        }
        const T* wt = w + ((int64_t)(a * 8 + e) * wcout + col) * cin_p + ci;
#pragma unroll
        for (int m = 0; m < 2; ++m) af[m] = P::load(wt + (int64_t)m * 16 * cin_p);
    };
    // one step of look-ahead: the next step's loads are in flight during this step's products
    Frag bcur[2], acur[2];
    if (s0 < s1) load_step(s0, bcur, acur);
    for (int st = s0; st < s1; ++st) {
        // the last step reloads its own fragments (unused): no branch around the loads, so the
        // wait for them can sit just before their first use
        Frag bnxt[2], anxt[2];
        load_step(st + 1 < s1 ? st + 1 : st, bnxt, anxt);
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int t = 0; t < 2; ++t) acc[m][t] = P::mma(acur[m], bcur[t], acc[m][t]);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            bcur[t] = bnxt[t];
            acur[t] = anxt[t];
        }
    }
    if (ks > 1) {
        // red[wave][16 values][64 lanes]: lane-fastest, conflict-free
        Acc* red = (Acc*)c8_smem;
        if (kw > 0) {
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) red[(wv * 16 + (m * 2 + t) * 4 + r) * 64 + lane] = acc[m][t][r];
        }
        __syncthreads();
        if (kw > 0) return;
        for (int j = 1; j < ks; ++j)
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[m][t][r] += red[((wv + j) * 16 + (m * 2 + t) * 4 + r) * 64 + lane];
    }
    const Acc slope = bias[COUT];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        if (!qv[t]) continue;
        const int oy = UP ? 2 * qy[t] + py : qy[t];
        const int ox = UP ? 2 * qx[t] + px : qx[t];
        const int64_t o = (((int64_t)b * Ho + oy) * Wo + ox) * COUT;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            Acc v[4], sv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const Acc s = acc[m][t][r] + bias[m * 16 + P::row_of(g, r)];
                sv[r] = s;
                v[r] = s > 0 ? s : slope * s;
            }
            store_rows<P>(y + o + m * 16 + P::row_of(g, 0), v);
            if (ypre) store_rows<P>(ypre + o + m * 16 + P::row_of(g, 0), sv);   // pre-activation (training)
        }
    }
}

template <class P>
int launch_conv8(bool up, const typename P::T* x0, const typename P::T* x1, int cin_p, int cat_cp,
                 const typename P::T* w, const typename P::Acc* bias, typename P::T* y, int cout_p, int Hin, int Win,
                 int batch, const int* skip, hipStream_t s, typename P::T* ypre, int wcout) {
    // shapes the kernel assumes: 32 output channels, input channels in whole K steps (a step of
    // 4 GW values may span several taps when cin_p < 4 GW), even input sides for the down form
    if (cout_p != 32 || cin_p < P::GW || cin_p % P::GW || cin_p > 64 || ((up ? 16 : 64) * cin_p) % (4 * P::GW) ||
        (cat_cp > 0 && (!x1 || cat_cp % P::GW || cat_cp >= cin_p)) || Hin < 1 || Win < 1 || batch < 1 ||
        (!up && (Hin % 2 || Win % 2)) || wcout < 32) {
        set_error("conv8: unsupported layer shape");
        return HZ_ERR_ARG;
    }
    const int64_t px = up ? (int64_t)Hin * Win : (int64_t)(Hin / 2) * (Win / 2);
    const int tiles = (int)((px + C8_PX - 1) / C8_PX);
    const int64_t items = (int64_t)batch * (up ? 4 : 1) * tiles;
    // split K over up to 8 wavefronts while the grid holds fewer than 2048 wavefronts (about 8 per
    // compute unit); the split depends on the sizes only, so results are reproducible
    const int nsteps = (up ? 16 : 64) * cin_p / (4 * P::GW);
    int ks = 1;
    while (ks < 8 && items * ks < 2048 && nsteps % (2 * ks) == 0) ks *= 2;
    const int nw = ks <= 4 ? 4 : 8;
    const int64_t per_block = nw / ks;
    const unsigned grid = (unsigned)((items + per_block - 1) / per_block);
    const size_t shm = ks > 1 ? (size_t)nw * 16 * 64 * sizeof(typename P::Acc) : 0;
    if (up)
        hipLaunchKernelGGL((k_conv8<P, true>), dim3(grid), dim3(64 * nw), shm, s, x0, x1, cin_p, cat_cp, w, bias, y,
                           Hin, Win, batch, tiles, ks, skip, ypre, wcout);
    else
        hipLaunchKernelGGL((k_conv8<P, false>), dim3(grid), dim3(64 * nw), shm, s, x0, x1, cin_p, cat_cp, w, bias, y,
                           Hin, Win, batch, tiles, ks, skip, ypre, wcout);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

template int launch_conv8<PolBF16>(bool, const bf16_t*, const bf16_t*, int, int, const bf16_t*, const float*, bf16_t*,
                                   int, int, int, int, const int*, hipStream_t, bf16_t*, int);
template int launch_conv8<PolF32>(bool, const float*, const float*, int, int, const float*, const float*, float*, int,
                                  int, int, int, const int*, hipStream_t, float*, int);
template int launch_conv8<PolF64>(bool, const double*, const double*, int, int, const double*, const double*, double*,
                                  int, int, int, int, const int*, hipStream_t, double*, int);

}  // namespace hz
