// Training step of the neural operator (Sections 3.3-3.4, eq. (10)-(12)): the
// physics-informed loss mean_b ||A_b N(r_b) - r_b|| / ||r_b|| (or its square), its
// gradient by reverse mode through the adjoint stencil and the U-Net, and Adam.
//
// Reverse mode, with G(layer) = d loss / d(pre-activation of the layer):
//   head:      g_out = coef_b s_b (A_b^H y_b) with y_b = r_b - A_b z_b and
//              coef_b = -1 / (B ||y_b|| ||r_b||) (squared: -2 / (B ||r_b||^2));
//              G(dec0b) = (g_out . W_head) masked by D0 > 0;
//   3x3 conv:  dW[co][ci][tap] = sum_p G[p][co] x[p + tap][ci], db = sum_p G;
//              d x = 3x3 convolution of G with the flipped, transposed weights (the forward
//              MFMA kernel with the data-gradient pack), masked by the producer's ReLU;
//   concat:    the data gradient splits into the skip part (E_l) and the up part (U_l);
//   transposed conv: dW[ab][co][ci] = sum_i G[2i + ab][co] x[i][ci]; d x = 2x2 stride-2
//              gather of G with the transposed weights (MFMA), masked by the input's ReLU;
//   pool:      G(enc_{l-1}b) = (skip + unpool(d P_l) / 4) masked by E_{l-1} > 0.
// Weight gradients accumulate in FP32 per pixel chunk and are summed over the chunks in a
// fixed order (deterministic).
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "krylov.h"
#include "krylov_impl.h"
#include "net_impl.h"
#include "problem.h"
#include "stencil_impl.h"

namespace hz {

constexpr int TT = 256;

// ------------------------------------------------------------------ pack / head (batched)

// s_b = ||r_b|| / sqrt(n) and ||r_b|| from per-sample norm partials (one wavefront per sample).
__global__ void k_sample_scales(const double2* part, int nblk, int64_t n, double* sc, double* nr) {
    const int b = blockIdx.x;
    double a = 0;
    for (int q = threadIdx.x; q < nblk; q += 64) a += part[(int64_t)b * nblk + q].x;
    a = wave_sum(a);
    if (threadIdx.x == 0) {
        const double s = sqrt(a / (double)n);
        sc[2 * b] = s;
        sc[2 * b + 1] = s > 0 ? 1.0 / s : 0.0;
        nr[b] = sqrt(a);
    }
}

// z_b = s_b (out_0 + i out_1) on the grid, out_k = sum_c D0[c] Wh[k][c] + bh[k].
template <class P>
__global__ void k_head_batched(const typename P::T* __restrict__ D, int cin_p, const typename P::T* __restrict__ wh,
                               const typename P::Acc* __restrict__ bh, const double* __restrict__ sc, int nxt,
                               int nyt, int Hp, int Wp, int B, float2* __restrict__ z) {
    using Acc = typename P::Acc;
    const int64_t n = (int64_t)nxt * nyt;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * B) return;
    const int b = (int)(idx / n);
    const int64_t g = idx - (int64_t)b * n;
    const int yy = (int)(g / nxt), xx = (int)(g % nxt);
    using T = typename P::T;
    constexpr int VE = 16 / sizeof(T);
    const T* d = D + (((int64_t)b * Hp + yy) * Wp + xx) * cin_p;
    Acc o0 = bh[0], o1 = bh[1];
    for (int c0 = 0; c0 < cin_p; c0 += VE) {   // 16-byte loads, channels summed in order
        const uint4 dv = *(const uint4*)(d + c0);
        const T* dd = (const T*)&dv;
#pragma unroll
        for (int k = 0; k < VE; ++k) {
            const Acc x = P::val(dd[k]);
            o0 += x * P::val(wh[c0 + k]);
            o1 += x * P::val(wh[cin_p + c0 + k]);
        }
    }
    const double s = sc[2 * b];
    z[idx] = float2{(float)(s * (double)o0), (float)(s * (double)o1)};
}

// Per-sample loss from the partials of ||y_b||^2 (y_b = r_b - A_b z_b) and ||r_b||; the
// head-gradient scale coef_b; the batch mean.
__global__ void k_loss(const double* __restrict__ ypart, int nparts, const double* __restrict__ nr, int B, int squared,
                       float* __restrict__ coef, float* __restrict__ loss, float* __restrict__ per_sample) {
    __shared__ double ls[1024];
    for (int b = threadIdx.x >> 6; b < B; b += blockDim.x >> 6) {
        double a = 0;
        for (int q = threadIdx.x & 63; q < nparts; q += 64) a += ypart[(int64_t)b * nparts + q];
        a = wave_sum(a);
        if ((threadIdx.x & 63) == 0) {
            const double nq = sqrt(a), r = nr[b];
            double l, cf;
            if (squared) {
                l = nq * nq / (r * r);
                cf = -2.0 / ((double)B * r * r);
            } else {
                l = nq / r;
                cf = nq > 0 ? -1.0 / ((double)B * nq * r) : 0.0;
            }
            ls[b] = l;
            coef[b] = (float)cf;
            if (per_sample) per_sample[b] = (float)l;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int b = 0; b < B; ++b) t += ls[b];
        *loss = (float)(t / B);
    }
}

// g_out at a padded pixel (0 off the grid).
__device__ inline float2 head_grad(const float2* gz, const float* coef, const double* sc, int b, int yy, int xx,
                                   int nxt, int nyt) {
    if (yy >= nyt || xx >= nxt) return float2{0.f, 0.f};
    const float2 a = gz[(int64_t)b * nxt * nyt + (int64_t)yy * nxt + xx];
    const float f = coef[b] * (float)sc[2 * b];
    return float2{f * a.x, f * a.y};
}

// G(dec0b)[p][c] = (g0 Wh[0][c] + g1 Wh[1][c]) masked by D0[p][c] > 0.
template <class P>
__global__ void k_head_dgrad(const float2* __restrict__ gz, const float* __restrict__ coef,
                             const double* __restrict__ sc, const typename P::T* __restrict__ D0, int cin_p,
                             const typename P::T* __restrict__ wh, int nxt, int nyt, int Hp, int Wp, int B,
                             typename P::T* __restrict__ G) {
    // one 16-byte vector of VE channels of one padded pixel per thread
    using T = typename P::T;
    using Acc = typename P::Acc;
    constexpr int VE = 16 / sizeof(T);
    const int nvec = cin_p / VE;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = (int64_t)Hp * Wp;
    if (idx >= np * B * nvec) return;
    const int c0 = (int)(idx % nvec) * VE;
    const int64_t pp = idx / nvec;
    const int b = (int)(pp / np);
    const int64_t q = pp - (int64_t)b * np;
    const float2 g = head_grad(gz, coef, sc, b, (int)(q / Wp), (int)(q % Wp), nxt, nyt);
    const uint4 dv = *(const uint4*)(D0 + pp * cin_p + c0);
    const T* d = (const T*)&dv;
    __attribute__((aligned(16))) T out[VE];
#pragma unroll
    for (int k = 0; k < VE; ++k) {
        Acc v = (Acc)g.x * P::val(wh[c0 + k]) + (Acc)g.y * P::val(wh[cin_p + c0 + k]);
        if (!(P::val(d[k]) > Acc(0))) v = Acc(0);
        out[k] = P::cvt(v);
    }
    *(uint4*)(G + pp * cin_p + c0) = *(const uint4*)out;
}

// Head weight / bias gradient partials: block z covers a slice of the padded pixels of all
// samples; part[z][k][c] = sum g_k D0[c] (c < cin_p), part[z][2][k] = sum g_k. A thread holds one
// 16-byte vector of VE channels of a pixel; the pixel lanes are summed in a fixed order.
template <class P>
__global__ void k_head_wgrad(const float2* __restrict__ gz, const float* __restrict__ coef,
                             const double* __restrict__ sc, const typename P::T* __restrict__ D0, int cin_p, int nxt,
                             int nyt, int Hp, int Wp, int B, int64_t per, float* __restrict__ part) {
    using T = typename P::T;
    constexpr int VE = 16 / sizeof(T);
    const int nvec = cin_p / VE;                        // vectors per pixel (divides 256)
    const int64_t np = (int64_t)Hp * Wp * B;
    const int64_t p0 = (int64_t)blockIdx.x * per, p1 = min(np, p0 + per);
    const int lanes = TT / nvec;                        // pixel lanes
    const int cv = threadIdx.x % nvec, pl = threadIdx.x / nvec;
    float a0[VE], a1[VE], s0 = 0, s1 = 0;
#pragma unroll
    for (int k = 0; k < VE; ++k) a0[k] = a1[k] = 0;
    for (int64_t p = p0 + pl; p < p1; p += lanes) {
        const int b = (int)(p / ((int64_t)Hp * Wp));
        const int64_t q = p - (int64_t)b * Hp * Wp;
        const float2 g = head_grad(gz, coef, sc, b, (int)(q / Wp), (int)(q % Wp), nxt, nyt);
        const uint4 dv = *(const uint4*)(D0 + p * cin_p + cv * VE);
        const T* d = (const T*)&dv;
#pragma unroll
        for (int k = 0; k < VE; ++k) {
            const float x = (float)P::val(d[k]);
            a0[k] += g.x * x;
            a1[k] += g.y * x;
        }
        s0 += g.x;
        s1 += g.y;
    }
    __shared__ float red[TT][2 * 8 + 2];
#pragma unroll
    for (int k = 0; k < VE; ++k) {
        red[threadIdx.x][k] = a0[k];
        red[threadIdx.x][8 + k] = a1[k];
    }
    red[threadIdx.x][16] = s0;
    red[threadIdx.x][17] = s1;
    __syncthreads();
    if (threadIdx.x < cin_p) {
        const int c = threadIdx.x, v = c / VE, k = c % VE;
        float t0 = 0, t1 = 0;
        for (int l = 0; l < lanes; ++l) {
            t0 += red[l * nvec + v][k];
            t1 += red[l * nvec + v][8 + k];
        }
        part[(int64_t)blockIdx.x * (2 * cin_p + 2) + c] = t0;
        part[(int64_t)blockIdx.x * (2 * cin_p + 2) + cin_p + c] = t1;
    }
    if (threadIdx.x == 0) {
        float t0 = 0, t1 = 0;
        for (int l = 0; l < lanes; ++l) {   // the vector-0 thread of every pixel lane saw each pixel once
            t0 += red[l * nvec][16];
            t1 += red[l * nvec][17];
        }
        part[(int64_t)blockIdx.x * (2 * cin_p + 2) + 2 * cin_p] = t0;
        part[(int64_t)blockIdx.x * (2 * cin_p + 2) + 2 * cin_p + 1] = t1;
    }
}

// One wavefront per output (2 cin weights, then 2 biases): lanes sum strided chunks, then a
// fixed-order wavefront sum.
__global__ void k_head_reduce(const float* __restrict__ part, int nchunk, int cin_p, Layer ly, float* __restrict__ grad) {
    const int t = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int ln = threadIdx.x & 63;
    const int nw = ly.cout * ly.cin;   // [2][cin]
    if (t >= nw + 2) return;
    const int slot = t < nw ? (t / ly.cin) * cin_p + t % ly.cin : 2 * cin_p + (t - nw);
    float a = 0;
    for (int z = ln; z < nchunk; z += 64) a += part[(int64_t)z * (2 * cin_p + 2) + slot];
    a = wave_sum(a);
    if (ln == 0) {
        if (t < nw) grad[ly.w_off + t] = a;
        else grad[ly.b_off + (t - nw)] = a;
    }
}

// ------------------------------------------------------------------ weight gradients

// 3x3: block (ci tile of 16, co tile of 16, chunk z) accumulates, over its 8 x 16 pixel tiles,
// dW[co][ci][tap] into part[z][co][ci][tap] and (ci tile 0) db[co] into partb[z][co].
template <class P>
__global__ __launch_bounds__(TT) void k_wgrad3(const typename P::T* __restrict__ G, int cout_p,
                                               const typename P::T* __restrict__ x0, int c0,
                                               const typename P::T* __restrict__ x1, int c1, int H, int W,
                                               int ntiles, int tpc, float* __restrict__ part,
                                               float* __restrict__ partb) {
    __shared__ float gs[128][17];
    __shared__ float xs[180][17];
    const int cin_p = c0 + c1;
    const int ci0 = blockIdx.x * 16, co0 = blockIdx.y * 16;
    const int z = blockIdx.z;
    const int tco = threadIdx.x >> 4, tci = threadIdx.x & 15;
    const int tx_n = (W + 15) / 16, ty_n = (H + 7) / 8;
    const int per_img = tx_n * ty_n;
    float acc[9], accb = 0;
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = 0;
    const int64_t plane = (int64_t)H * W;
    const int t_end = min(ntiles, (z + 1) * tpc);
    for (int tile = z * tpc; tile < t_end; ++tile) {
        const int b = tile / per_img, r = tile - b * per_img;
        const int ty0 = (r / tx_n) * 8, tx0 = (r % tx_n) * 16;
        __syncthreads();
        for (int v = threadIdx.x; v < 128 * 16; v += TT) {
            const int px = v >> 4, c = v & 15;
            const int gy = ty0 + (px >> 4), gx = tx0 + (px & 15);
            float val = 0.f;
            if (gy < H && gx < W) val = (float)P::val(G[((int64_t)b * plane + (int64_t)gy * W + gx) * cout_p + co0 + c]);
            gs[px][c] = val;
        }
        for (int v = threadIdx.x; v < 180 * 16; v += TT) {
            const int px = v >> 4, c = v & 15;
            const int gy = ty0 + px / 18 - 1, gx = tx0 + px % 18 - 1;
            const int ci = ci0 + c;
            float val = 0.f;
            if (gy >= 0 && gy < H && gx >= 0 && gx < W && ci < cin_p) {
                const int64_t pix = (int64_t)b * plane + (int64_t)gy * W + gx;
                val = (float)P::val(ci < c0 ? x0[pix * c0 + ci] : x1[pix * c1 + ci - c0]);
            }
            xs[px][c] = val;
        }
        __syncthreads();
        for (int px = 0; px < 128; ++px) {
            const float g = gs[px][tco];
            const int py = px >> 4, pxx = px & 15;
#pragma unroll
            for (int t = 0; t < 9; ++t) acc[t] += g * xs[(py + t / 3) * 18 + pxx + t % 3][tci];
            accb += g;
        }
    }
    const int co = co0 + tco, ci = ci0 + tci;
    if (ci < cin_p) {
        float* dst = part + (((int64_t)z * cout_p + co) * cin_p + ci) * 9;
#pragma unroll
        for (int t = 0; t < 9; ++t) dst[t] = acc[t];
    }
    if (blockIdx.x == 0 && tci == 0) partb[(int64_t)z * cout_p + co] = accb;
}

// 8 x 8 transpose of 16-bit elements: r[p] holds elements 0..7 of row p; o[k] receives element k
// of rows 0..7 (row p in its element p)
__device__ __forceinline__ void wg_transpose8(const uint4 (&r)[8], uint4 (&o)[8]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        uint32_t wv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t a = (&r[2 * j].x)[k >> 1], c = (&r[2 * j + 1].x)[k >> 1];
            wv[j] = (k & 1) ? ((a >> 16) | (c & 0xffff0000u)) : ((a & 0xffffu) | (c << 16));
        }
        o[k] = uint4{wv[0], wv[1], wv[2], wv[3]};
    }
}

// 3x3 on the matrix cores (BF16 operands, FP32 accumulation): for every tap (dy, dx),
// dW[co][ci][tap] = sum_p G[p][co] X[p + (dy - 1, dx - 1)][ci] is a product with the pixels as
// the reduction index. Block: 32 output x 32 input channels over its chunk of 8 x 16 pixel
// tiles. Each tile is staged in LDS transposed (pixels contiguous per channel) so that a lane's
// 8 consecutive reduction elements are one 16-byte read; the input patch is stored three times,
// shifted by dx, to keep those reads aligned. Wavefront w owns the 16 x 16 channel pair
// (w / 2, w % 2) for all 9 taps. Partials and bias sums as in k_wgrad3.
constexpr int WG_CO = 32, WG_CI = 32;
constexpr int WG_GS = 128 + 8;              // LDS row of Gt: 128 pixels (+16 B)
constexpr int WG_XS = 10 * 16 + 8;          // LDS plane of one channel of Xt: 10 rows x 16 (+16 B)

__global__ __launch_bounds__(TT) void k_wgrad3_mfma(const bf16_t* __restrict__ G, int cout_p,
                                                    const bf16_t* __restrict__ x0, int c0,
                                                    const bf16_t* __restrict__ x1, int c1, int H, int W,
                                                    int ntiles, int tpc, float* __restrict__ part,
                                                    float* __restrict__ partb) {
    __shared__ __attribute__((aligned(16))) bf16_t gt[WG_CO * WG_GS];
    __shared__ __attribute__((aligned(16))) bf16_t xt[3 * WG_CI * WG_XS];
    const int cin_p = c0 + c1;
    const int ci0 = blockIdx.x * WG_CI, co0 = blockIdx.y * WG_CO;
    const int z = blockIdx.z;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, kg = lane >> 4;
    const int cob = wv >> 1, cib = wv & 1;
    const int tx_n = (W + 15) / 16, ty_n = (H + 7) / 8;
    const int per_img = tx_n * ty_n;
    const int64_t plane = (int64_t)H * W;
    f32x4_t acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][r] = 0.f;
    float accb = 0.f;                            // bias: thread sums 16 pixels of channel threadIdx.x / 8
    const int t_beg = z * tpc, t_end = min(ntiles, (z + 1) * tpc);
    // G tile (128 pixels x 32 channels) and the three shifted copies of the input patch, staged
    // transposed: a thread loads its unit's pixel vectors into registers (the next tile's while the
    // matrix cores work on this one), transposes 8 pixels x 8 channels at a time (wg_transpose8)
    // and writes 8 channel rows of 8 pixels as 16-byte stores (the same LDS contents as
    // element-wise transposing stores). Units [0, 64): G, 8 pixels; [64, 144): 10 pixels of one
    // patch row (columns 8 h .. 8 h + 9), from which the three copies take their 8-pixel windows.
    constexpr int NU = 16 * 4 + 10 * 2 * 4;
    static_assert(NU <= TT, "one unit per thread");
    uint4 rg[10];
    auto gload = [&](int tile) {
        const int b = tile / per_img, r = tile - b * per_img;
        const int ty0 = (r / tx_n) * 8, tx0 = (r % tx_n) * 16;
        const int u = threadIdx.x;
        if (u >= NU) return;
        const int part8 = u & 3;
        if (u < 16 * 4) {   // G: pixels 8 pg .. 8 pg + 7 of the tile (row pg / 2, columns 8 (pg % 2) ..)
            const int pg = u >> 2;
            const int gy = ty0 + (pg >> 1), gx0 = tx0 + 8 * (pg & 1);
            const int co = co0 + part8 * 8;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                rg[k] = uint4{0, 0, 0, 0};
                if (gy < H && gx0 + k < W && co < cout_p)
                    rg[k] = *(const uint4*)(G + ((int64_t)b * plane + (int64_t)gy * W + gx0 + k) * cout_p + co);
            }
        } else {            // X: patch row py, patch columns 8 h .. 8 h + 9
            const int q = u - 16 * 4;
            const int h = (q >> 2) & 1, py = q >> 3;
            const int gy = ty0 + py - 1, gx0 = tx0 + 8 * h - 1;
            const int ci = ci0 + part8 * 8;
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                const int gx = gx0 + k;
                rg[k] = uint4{0, 0, 0, 0};
                if (gy >= 0 && gy < H && gx >= 0 && gx < W && ci < cin_p) {
                    const int64_t pix = (int64_t)b * plane + (int64_t)gy * W + gx;
                    rg[k] = *(const uint4*)(ci < c0 ? x0 + pix * c0 + ci : x1 + pix * c1 + (ci - c0));
                }
            }
        }
    };
    auto put = [&](bf16_t* dst, int stride, int off) {   // the 8 pixels rg[off ..] transposed to dst
        uint4 w8[8], o[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) w8[k] = rg[off + k];
        wg_transpose8(w8, o);
#pragma unroll
        for (int k = 0; k < 8; ++k) *(uint4*)(dst + k * stride) = o[k];
    };
    auto lstore = [&]() {
        const int u = threadIdx.x;
        if (u >= NU) return;
        const int part8 = u & 3;
        if (u < 16 * 4) {
            put(&gt[(part8 * 8) * WG_GS + 8 * (u >> 2)], WG_GS, 0);
        } else {            // copy dx, columns 8 h .. 8 h + 7 hold patch columns 8 h + dx ..
            const int q = u - 16 * 4;
            const int h = (q >> 2) & 1, py = q >> 3;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
                put(&xt[(dx * WG_CI + part8 * 8) * WG_XS + py * 16 + 8 * h], WG_XS, dx);
        }
    };
    if (t_beg < t_end) gload(t_beg);
    for (int tile = t_beg; tile < t_end; ++tile) {
        __syncthreads();   // the previous tile's reads of the LDS are done
        lstore();
        __syncthreads();
        if (tile + 1 < t_end) gload(tile + 1);
        if (blockIdx.x == 0) {
            const int co = threadIdx.x >> 3, seg = threadIdx.x & 7;
#pragma unroll
            for (int k = 0; k < 16; ++k) accb += bf2f(gt[co * WG_GS + seg * 16 + k]);
        }
        // 4 reduction steps of 32 pixels (step s: tile rows 2s, 2s + 1), every tap's accumulator
        // taking the steps in order. The input fragment of step s and row offset dy starts at patch
        // row 2s + dy: per column offset dx, the 9 distinct fragments are read once for all steps.
        bf16x8_t a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] = PolBF16::load(&gt[(cob * 16 + lr) * WG_GS + 32 * s + 8 * kg]);
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            bf16x8_t bq[9];
#pragma unroll
            for (int q = 0; q < 9; ++q)
                bq[q] = PolBF16::load(&xt[(dx * WG_CI + cib * 16 + lr) * WG_XS + (q + (kg >> 1)) * 16 + 8 * (kg & 1)]);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) acc[dy * 3 + dx] = PolBF16::mma(a[s], bq[2 * s + dy], acc[dy * 3 + dx]);
        }
    }
    // lane holds D[co = co0 + 16 cob + 4 kg + r][ci = ci0 + 16 cib + lr] of every tap
    const int ci = ci0 + cib * 16 + lr;
    if (ci < cin_p) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = co0 + cob * 16 + 4 * kg + r;
            if (co < cout_p) {
                float* dst = part + (((int64_t)z * cout_p + co) * cin_p + ci) * 9;
#pragma unroll
                for (int t = 0; t < 9; ++t) dst[t] = acc[t][r];
            }
        }
    }
    if (blockIdx.x == 0) {
        accb += __shfl_xor(accb, 1, 64);
        accb += __shfl_xor(accb, 2, 64);
        accb += __shfl_xor(accb, 4, 64);
        const int co = co0 + (threadIdx.x >> 3);
        if ((threadIdx.x & 7) == 0 && co < cout_p) partb[(int64_t)z * cout_p + co] = accb;
    }
}

// The same product in FP32 on the matrix cores (v_mfma_f32_16x16x4_f32: one reduction element
// per lane, 4 pixels per instruction). Block, tiles, partials and bias sums as in k_wgrad3_mfma;
// the transposed LDS copies hold FP32 values, and a single copy of the 10 x 18 input patch serves
// every dx since a lane reads one value. Row pitches of 130 and 194 floats (2 mod 32) make the 32
// lanes of a half-wavefront hit 32 distinct banks.
constexpr int WF_GS = 128 + 2;
constexpr int WF_XS = 10 * 18 + 14;

__global__ __launch_bounds__(TT) void k_wgrad3_mfma_f32(const float* __restrict__ G, int cout_p,
                                                        const float* __restrict__ x0, int c0,
                                                        const float* __restrict__ x1, int c1, int H, int W,
                                                        int ntiles, int tpc, float* __restrict__ part,
                                                        float* __restrict__ partb) {
    __shared__ float gt[WG_CO * WF_GS];
    __shared__ float xt[WG_CI * WF_XS];
    const int cin_p = c0 + c1;
    const int ci0 = blockIdx.x * WG_CI, co0 = blockIdx.y * WG_CO;
    const int z = blockIdx.z;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, kg = lane >> 4;
    const int cob = wv >> 1, cib = wv & 1;
    const int tx_n = (W + 15) / 16, ty_n = (H + 7) / 8;
    const int per_img = tx_n * ty_n;
    const int64_t plane = (int64_t)H * W;
    f32x4_t acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][r] = 0.f;
    float accb = 0.f;
    const int t_beg = z * tpc, t_end = min(ntiles, (z + 1) * tpc);
    // G tile (128 pixels x 32 channels) and input patch (10 x 18 pixels x 32 channels) as vectors
    // of 4 channels: a thread's vectors of the next tile are loaded into registers while the
    // matrix cores work on this one, then written transposed (one value per LDS row)
    constexpr int NGV = (128 * 8 + TT - 1) / TT, NXV = (180 * 8 + TT - 1) / TT;
    float4 rgv[NGV], rxv[NXV];
    auto gload = [&](int tile) {
        const int b = tile / per_img, r = tile - b * per_img;
        const int ty0 = (r / tx_n) * 8, tx0 = (r % tx_n) * 16;
#pragma unroll
        for (int i = 0; i < NGV; ++i) {
            const int v = threadIdx.x + i * TT;
            const int px = v >> 3, part4 = v & 7;
            const int gy = ty0 + (px >> 4), gx = tx0 + (px & 15);
            const int co = co0 + part4 * 4;
            rgv[i] = float4{0.f, 0.f, 0.f, 0.f};
            if (v < 128 * 8 && gy < H && gx < W && co < cout_p)
                rgv[i] = *(const float4*)(G + ((int64_t)b * plane + (int64_t)gy * W + gx) * cout_p + co);
        }
#pragma unroll
        for (int i = 0; i < NXV; ++i) {
            const int v = threadIdx.x + i * TT;
            const int px = v >> 3, part4 = v & 7;
            const int py = px / 18, pc = px - py * 18;
            const int gy = ty0 + py - 1, gx = tx0 + pc - 1;
            const int ci = ci0 + part4 * 4;
            rxv[i] = float4{0.f, 0.f, 0.f, 0.f};
            if (v < 180 * 8 && gy >= 0 && gy < H && gx >= 0 && gx < W && ci < cin_p) {
                const int64_t pix = (int64_t)b * plane + (int64_t)gy * W + gx;
                rxv[i] = *(const float4*)(ci < c0 ? x0 + pix * c0 + ci : x1 + pix * c1 + (ci - c0));
            }
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int i = 0; i < NGV; ++i) {
            const int v = threadIdx.x + i * TT;
            if (v < 128 * 8) {
                const int px = v >> 3, part4 = v & 7;
                gt[(part4 * 4 + 0) * WF_GS + px] = rgv[i].x;
                gt[(part4 * 4 + 1) * WF_GS + px] = rgv[i].y;
                gt[(part4 * 4 + 2) * WF_GS + px] = rgv[i].z;
                gt[(part4 * 4 + 3) * WF_GS + px] = rgv[i].w;
            }
        }
#pragma unroll
        for (int i = 0; i < NXV; ++i) {
            const int v = threadIdx.x + i * TT;
            if (v < 180 * 8) {
                const int px = v >> 3, part4 = v & 7;
                xt[(part4 * 4 + 0) * WF_XS + px] = rxv[i].x;
                xt[(part4 * 4 + 1) * WF_XS + px] = rxv[i].y;
                xt[(part4 * 4 + 2) * WF_XS + px] = rxv[i].z;
                xt[(part4 * 4 + 3) * WF_XS + px] = rxv[i].w;
            }
        }
    };
    if (t_beg < t_end) gload(t_beg);
    for (int tile = t_beg; tile < t_end; ++tile) {
        __syncthreads();   // the previous tile's reads of the LDS are done
        lstore();
        __syncthreads();
        if (tile + 1 < t_end) gload(tile + 1);
        if (blockIdx.x == 0) {
            const int co = threadIdx.x >> 3, seg = threadIdx.x & 7;
#pragma unroll
            for (int k = 0; k < 16; ++k) accb += gt[co * WF_GS + seg * 16 + k];
        }
        // 32 reduction steps of 4 pixels: lane group kg takes pixel 4 q + kg
#pragma unroll 4
        for (int q = 0; q < 32; ++q) {
            const int p = 4 * q + kg;
            const int row = p >> 4, col = p & 15;
            const float a = gt[(cob * 16 + lr) * WF_GS + p];
            const float* xb = &xt[(cib * 16 + lr) * WF_XS + row * 18 + col];
#pragma unroll
            for (int t = 0; t < 9; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, xb[(t / 3) * 18 + t % 3], acc[t], 0, 0, 0);
        }
    }
    // lane holds D[co = co0 + 16 cob + 4 kg + r][ci = ci0 + 16 cib + lr] of every tap
    const int ci = ci0 + cib * 16 + lr;
    if (ci < cin_p) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = co0 + cob * 16 + 4 * kg + r;
            if (co < cout_p) {
                float* dst = part + (((int64_t)z * cout_p + co) * cin_p + ci) * 9;
#pragma unroll
                for (int t = 0; t < 9; ++t) dst[t] = acc[t][r];
            }
        }
    }
    if (blockIdx.x == 0) {
        accb += __shfl_xor(accb, 1, 64);
        accb += __shfl_xor(accb, 2, 64);
        accb += __shfl_xor(accb, 4, 64);
        const int co = co0 + (threadIdx.x >> 3);
        if ((threadIdx.x & 7) == 0 && co < cout_p) partb[(int64_t)z * cout_p + co] = accb;
    }
}

// Transposed 2x2: dW[ab][co][ci] = sum_i G[2i + ab][co] x[i][ci]; block: ci tile, co tile, chunk of
// 8 x 8 input tiles.
template <class P>
__global__ __launch_bounds__(TT) void k_wgradT(const typename P::T* __restrict__ G, int cout_p,
                                               const typename P::T* __restrict__ x, int cin_p, int H, int W,
                                               int ntiles, int tpc, float* __restrict__ part,
                                               float* __restrict__ partb) {
    __shared__ float gs[64][4][17];
    __shared__ float xs[64][17];
    const int ci0 = blockIdx.x * 16, co0 = blockIdx.y * 16;
    const int z = blockIdx.z;
    const int tco = threadIdx.x >> 4, tci = threadIdx.x & 15;
    const int tx_n = (W + 7) / 8, ty_n = (H + 7) / 8;
    const int per_img = tx_n * ty_n;
    float acc[4] = {0, 0, 0, 0}, accb = 0;
    const int64_t plane = (int64_t)H * W;
    const int t_end = min(ntiles, (z + 1) * tpc);
    for (int tile = z * tpc; tile < t_end; ++tile) {
        const int b = tile / per_img, r = tile - b * per_img;
        const int ty0 = (r / tx_n) * 8, tx0 = (r % tx_n) * 8;
        __syncthreads();
        for (int v = threadIdx.x; v < 64 * 4 * 16; v += TT) {
            const int c = v & 15, ab = (v >> 4) & 3, px = v >> 6;
            const int iy = ty0 + (px >> 3), ix = tx0 + (px & 7);
            float val = 0.f;
            if (iy < H && ix < W) {
                const int oy = 2 * iy + (ab >> 1), ox = 2 * ix + (ab & 1);
                val = (float)P::val(G[((int64_t)b * 4 * plane + (int64_t)oy * 2 * W + ox) * cout_p + co0 + c]);
            }
            gs[px][ab][c] = val;
        }
        for (int v = threadIdx.x; v < 64 * 16; v += TT) {
            const int c = v & 15, px = v >> 4;
            const int iy = ty0 + (px >> 3), ix = tx0 + (px & 7);
            float val = 0.f;
            if (iy < H && ix < W) val = (float)P::val(x[((int64_t)b * plane + (int64_t)iy * W + ix) * cin_p + ci0 + c]);
            xs[px][c] = val;
        }
        __syncthreads();
        for (int px = 0; px < 64; ++px) {
            const float xv = xs[px][tci];
#pragma unroll
            for (int ab = 0; ab < 4; ++ab) acc[ab] += gs[px][ab][tco] * xv;
            accb += gs[px][0][tco] + gs[px][1][tco] + gs[px][2][tco] + gs[px][3][tco];
        }
    }
    const int co = co0 + tco, ci = ci0 + tci;
    float* dst = part + (((int64_t)z * cout_p + co) * cin_p + ci) * 4;
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) dst[ab] = acc[ab];
    if (blockIdx.x == 0 && tci == 0) partb[(int64_t)z * cout_p + co] = accb;
}

// Transposed 2x2 on the matrix cores: for every output parity ab, dW[ab][co][ci] =
// sum_i G[2i + ab][co] x[i][ci] with the coarse pixels i as the reduction index. Block: 32 x 32
// channels over its chunk of 8 x 16 coarse tiles, staged transposed in LDS as in k_wgrad3_mfma;
// wavefront w owns the channel pair (w / 2, w % 2) for the 4 parities.
__global__ __launch_bounds__(TT) void k_wgradT_mfma(const bf16_t* __restrict__ G, int cout_p,
                                                    const bf16_t* __restrict__ x, int cin_p, int H, int W,
                                                    int ntiles, int tpc, float* __restrict__ part,
                                                    float* __restrict__ partb) {
    __shared__ __attribute__((aligned(16))) bf16_t gt[4 * WG_CO * WG_GS];
    __shared__ __attribute__((aligned(16))) bf16_t xt[WG_CI * WG_GS];
    const int ci0 = blockIdx.x * WG_CI, co0 = blockIdx.y * WG_CO;
    const int z = blockIdx.z;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, kg = lane >> 4;
    const int cob = wv >> 1, cib = wv & 1;
    const int tx_n = (W + 15) / 16, ty_n = (H + 7) / 8;
    const int per_img = tx_n * ty_n;
    const int64_t plane = (int64_t)H * W;
    f32x4_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][r] = 0.f;
    float accb = 0.f;
    const int t_beg = z * tpc, t_end = min(ntiles, (z + 1) * tpc);
    // G at the 4 fine pixels (parity ab) of each of the 128 coarse pixels, and x, staged transposed
    // by units of 8 coarse pixels x 8 channels as in k_wgrad3_mfma (register transposes, 16-byte
    // LDS stores, the next tile's loads in flight). Units [0, 256): G (ab, pixel group, part);
    // [256, 320): x.
    constexpr int NU = 4 * 16 * 4 + 16 * 4;
    constexpr int UPT = (NU + TT - 1) / TT;
    uint4 rg[UPT][8];
    auto gload = [&](int tile) {
        const int b = tile / per_img, r = tile - b * per_img;
        const int ty0 = (r / tx_n) * 8, tx0 = (r % tx_n) * 16;
#pragma unroll
        for (int i = 0; i < UPT; ++i) {
            const int u = threadIdx.x + i * TT;
            if (u >= NU) break;
            const int part8 = u & 3;
            const int pg = (u >> 2) & 15;
            const int iy = ty0 + (pg >> 1), ix0 = tx0 + 8 * (pg & 1);
            if (u < 4 * 16 * 4) {
                const int ab = u >> 6;
                const int co = co0 + part8 * 8;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    rg[i][k] = uint4{0, 0, 0, 0};
                    if (iy < H && ix0 + k < W && co < cout_p) {
                        const int oy = 2 * iy + (ab >> 1), ox = 2 * (ix0 + k) + (ab & 1);
                        rg[i][k] = *(const uint4*)(G + ((int64_t)b * 4 * plane + (int64_t)oy * 2 * W + ox) * cout_p + co);
                    }
                }
            } else {
                const int ci = ci0 + part8 * 8;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    rg[i][k] = uint4{0, 0, 0, 0};
                    if (iy < H && ix0 + k < W && ci < cin_p)
                        rg[i][k] = *(const uint4*)(x + ((int64_t)b * plane + (int64_t)iy * W + ix0 + k) * cin_p + ci);
                }
            }
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int i = 0; i < UPT; ++i) {
            const int u = threadIdx.x + i * TT;
            if (u >= NU) break;
            const int part8 = u & 3;
            const int pg = (u >> 2) & 15;
            bf16_t* dst = u < 4 * 16 * 4 ? &gt[((u >> 6) * WG_CO + part8 * 8) * WG_GS + 8 * pg]
                                         : &xt[(part8 * 8) * WG_GS + 8 * pg];
            uint4 o[8];
            wg_transpose8(rg[i], o);
#pragma unroll
            for (int k = 0; k < 8; ++k) *(uint4*)(dst + k * WG_GS) = o[k];
        }
    };
    if (t_beg < t_end) gload(t_beg);
    for (int tile = t_beg; tile < t_end; ++tile) {
        __syncthreads();   // the previous tile's reads of the LDS are done
        lstore();
        __syncthreads();
        if (tile + 1 < t_end) gload(tile + 1);
        if (blockIdx.x == 0) {
            const int co = threadIdx.x >> 3, seg = threadIdx.x & 7;
#pragma unroll
            for (int ab = 0; ab < 4; ++ab)
#pragma unroll
                for (int k = 0; k < 16; ++k) accb += bf2f(gt[(ab * WG_CO + co) * WG_GS + seg * 16 + k]);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bf16x8_t bb = PolBF16::load(&xt[(cib * 16 + lr) * WG_GS + 32 * s + 8 * kg]);
#pragma unroll
            for (int ab = 0; ab < 4; ++ab) {
                const bf16x8_t a = PolBF16::load(&gt[(ab * WG_CO + cob * 16 + lr) * WG_GS + 32 * s + 8 * kg]);
                acc[ab] = PolBF16::mma(a, bb, acc[ab]);
            }
        }
    }
    const int ci = ci0 + cib * 16 + lr;
    if (ci < cin_p) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = co0 + cob * 16 + 4 * kg + r;
            if (co < cout_p) {
                float* dst = part + (((int64_t)z * cout_p + co) * cin_p + ci) * 4;
#pragma unroll
                for (int ab = 0; ab < 4; ++ab) dst[ab] = acc[ab][r];
            }
        }
    }
    if (blockIdx.x == 0) {
        accb += __shfl_xor(accb, 1, 64);
        accb += __shfl_xor(accb, 2, 64);
        accb += __shfl_xor(accb, 4, 64);
        const int co = co0 + (threadIdx.x >> 3);
        if ((threadIdx.x & 7) == 0 && co < cout_p) partb[(int64_t)z * cout_p + co] = accb;
    }
}

// Sum the chunk partials of one layer into the flat FP32 gradient (logical channels).
// grad[...] = sum over the nchunk partials, in a fixed order: a block covers 32 consecutive
// outputs; thread group g (of 8) sums the chunks z = g mod 8, and the 8 group sums are added
// in order g = 0..7.
constexpr int WR_OUT = 32, WR_GRP = 8;
__global__ __launch_bounds__(WR_OUT * WR_GRP) void k_wgrad_reduce(const float* __restrict__ part,
                                                                 const float* __restrict__ partb, int nchunk,
                                                                 Layer ly, float* __restrict__ grad) {
    __shared__ float red[WR_GRP][WR_OUT];
    const int o = threadIdx.x % WR_OUT, g = threadIdx.x / WR_OUT;
    const int64_t t = (int64_t)blockIdx.x * WR_OUT + o;
    const int taps = ly.kind == L_CONV3 ? 9 : 4;
    const int64_t nw = (int64_t)taps * ly.cin * ly.cout;
    float a = 0;
    if (t < nw) {
        int co, ci, tap;
        if (ly.kind == L_CONV3) {         // flat [co][ci][tap]
            tap = (int)(t % 9);
            ci = (int)((t / 9) % ly.cin);
            co = (int)(t / (9 * ly.cin));
        } else {                          // flat [ci][co][ab]
            tap = (int)(t % 4);
            co = (int)((t / 4) % ly.cout);
            ci = (int)(t / (4 * ly.cout));
        }
        int cis = ci;                     // stored channel of a concatenated input
        if (ly.cat_cp > 0 && ci >= ly.cat_c) cis = ly.cat_cp + (ci - ly.cat_c);
        for (int z = g; z < nchunk; z += WR_GRP)
            a += part[(((int64_t)z * ly.cout_p + co) * ly.cin_p + cis) * taps + tap];
    } else if (t < nw + ly.cout) {
        const int co = (int)(t - nw);
        for (int z = g; z < nchunk; z += WR_GRP) a += partb[(int64_t)z * ly.cout_p + co];
    }
    red[g][o] = a;
    __syncthreads();
    if (g == 0 && t < nw + ly.cout) {
        float sum = 0;
#pragma unroll
        for (int k = 0; k < WR_GRP; ++k) sum += red[k][o];
        if (t < nw) grad[ly.w_off + t] = sum;
        else grad[ly.b_off + (t - nw)] = sum;
    }
}

// ------------------------------------------------------------------ data gradients

// Transposed-conv data gradient: gx[i][ci] = sum_{ab, co} G[2i + ab][co] Wt[ab][ci][co], masked by
// x[i][ci] > 0. Block: 64 input pixels of one row, TN input channels; K = (ab, co) chunks.
template <class P, int TN>
__global__ __launch_bounds__(TT) void k_convT2_dgrad(const typename P::T* __restrict__ G, int cout_p,
                                                     const typename P::T* __restrict__ wt,
                                                     const typename P::T* __restrict__ xmask,
                                                     typename P::T* __restrict__ gx, int cin_p, int H, int W, int ck) {
    using T = typename P::T;
    using AccV = typename P::AccV;
    using Frag = typename P::Frag;
    constexpr int PS = P::CK + 16 / (int)sizeof(T);
    constexpr int VE = 16 / sizeof(T);
    constexpr int NCB = TN / 16;
    __shared__ __attribute__((aligned(16))) T gl[64 * 4 * PS];
    __shared__ __attribute__((aligned(16))) T wl[4 * TN * PS];
    const int ncb_tot = cin_p / TN;
    const int bz = blockIdx.z / ncb_tot;
    const int ci0 = (blockIdx.z - bz * ncb_tot) * TN;
    const int iy = blockIdx.y, ix0 = blockIdx.x * 64;
    const int64_t plane = (int64_t)H * W;
    const T* gs = G + (int64_t)bz * plane * 4 * cout_p;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    AccV acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[cb][r] = 0;
    const int vpp = ck / VE;
    const int groups = ck / P::GW;
    const int steps = (groups + 3) / 4;
    for (int k0 = 0; k0 < cout_p; k0 += ck) {
        __syncthreads();
        for (int v = threadIdx.x; v < 64 * 4 * vpp; v += TT) {
            const int part = v % vpp, ab = (v / vpp) & 3, px = v / (4 * vpp);
            const int ix = ix0 + px;
            uint4 val = uint4{0, 0, 0, 0};
            if (ix < W) {
                const int oy = 2 * iy + (ab >> 1), ox = 2 * ix + (ab & 1);
                val = *(const uint4*)(gs + ((int64_t)oy * 2 * W + ox) * cout_p + k0 + part * VE);
            }
            *(uint4*)&gl[(px * 4 + ab) * PS + part * VE] = val;
        }
        for (int v = threadIdx.x; v < 4 * TN * vpp; v += TT) {
            const int part = v % vpp, row = v / vpp;
            const int ab = row / TN, ci = row - ab * TN;
            *(uint4*)&wl[row * PS + part * VE] =
                *(const uint4*)(wt + ((int64_t)ab * cin_p + ci0 + ci) * cout_p + k0 + part * VE);
        }
        __syncthreads();
        for (int st = 0; st < steps; ++st) {
            const int cg = 4 * st + lg;
#pragma unroll
            for (int ab = 0; ab < 4; ++ab) {
                const Frag b = cg < groups ? P::load(&gl[((wv * 16 + lr) * 4 + ab) * PS + cg * P::GW]) : P::zero();
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    const Frag a = cg < groups ? P::load(&wl[(ab * TN + cb * 16 + lr) * PS + cg * P::GW]) : P::zero();
                    acc[cb] = P::mma(a, b, acc[cb]);
                }
            }
        }
    }
    const int ix = ix0 + wv * 16 + lr;
    if (ix >= W) return;
    const int64_t pix = (int64_t)bz * plane + (int64_t)iy * W + ix;
    if constexpr (std::is_same<P, PolBF16>::value) {
        // a lane's 4 registers are 4 consecutive channels: one 8-byte mask load and one store
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int64_t o = pix * cin_p + ci0 + cb * 16 + P::row_of(lg, 0);
            const uint2 mk = *(const uint2*)(xmask + o);
            typename P::Acc v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t mw = r < 2 ? mk.x : mk.y;
                const T m = (T)((mw >> (16 * (r & 1))) & 0xffffu);
                v[r] = P::val(m) > typename P::Acc(0) ? acc[cb][r] : typename P::Acc(0);
            }
            store_rows<P>(gx + o, v);
        }
    } else {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ci = ci0 + cb * 16 + P::row_of(lg, r);
                typename P::Acc v = acc[cb][r];
                if (!(P::val(xmask[pix * cin_p + ci]) > typename P::Acc(0))) v = 0;
                gx[pix * cin_p + ci] = P::cvt(v);
            }
    }
}

// G(enc_{l-1}b) = (skip + unpool(dP) / 4) masked by E > 0, in place in skip. E, skip: [B][H][W][c];
// dP: [B][H/2][W/2][c].
template <class P>
__global__ void k_pool_bwd(typename P::T* __restrict__ skip, const typename P::T* __restrict__ dP,
                           const typename P::T* __restrict__ E, int H, int W, int c, int64_t total) {
    // one 16-byte vector of VE channels per thread (c is a multiple of 16)
    using T = typename P::T;
    using Acc = typename P::Acc;
    constexpr int VE = 16 / sizeof(T);
    const int64_t iv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (iv * VE >= total) return;
    const int64_t idx = iv * VE;
    const int ch = (int)(idx % c);
    const int64_t pp = idx / c;
    const int64_t plane = (int64_t)H * W;
    const int b = (int)(pp / plane);
    const int64_t q = pp - (int64_t)b * plane;
    const int yy = (int)(q / W), xx = (int)(q % W);
    const int64_t pi = ((int64_t)b * (plane / 4) + (int64_t)(yy / 2) * (W / 2) + xx / 2) * c + ch;
    const uint4 sv = *(const uint4*)(skip + idx), pv = *(const uint4*)(dP + pi), ev = *(const uint4*)(E + idx);
    const T *sk = (const T*)&sv, *pd = (const T*)&pv, *e = (const T*)&ev;
    __attribute__((aligned(16))) T out[VE];
#pragma unroll
    for (int k = 0; k < VE; ++k) {
        Acc v = P::val(sk[k]) + Acc(0.25) * P::val(pd[k]);
        if (!(P::val(e[k]) > Acc(0))) v = Acc(0);
        out[k] = P::cvt(v);
    }
    *(uint4*)(skip + idx) = *(const uint4*)out;
}

// ------------------------------------------------------------------ workspace

// The per-sample problem data a batched launch reads (every sample of a batch has the same grid).
struct SampleProb {
    const float* k2;
    const double *cnd, *sigx, *sigy;
    const float2 *fE, *fW, *fN, *fS, *aE, *aW, *aN, *aS, *dx, *dy;
};

template <class P>
struct TrainBufs {
    using T = typename P::T;
    FwdBufs f;                       // forward activations (kept for the backward)
    std::vector<T*> gA, gB, gU, gP;  // activation gradients per level
    float2 *z, *y, *gz;              // [B][n]
    double2* rpart;                  // [B][nblk] ||r_b||^2 partials
    double* ypart;                   // [B][stencil blocks] ||y_b||^2 partials
    double *sc, *nr;                 // [B][2], [B]
    float* coef;                     // [B]
    SampleProb* sprob;               // [B] per-sample problem pointers
    float *wpart, *wpartb;           // weight-gradient chunk partials
    size_t wcap, bcap;               // their capacities (floats)
    size_t total;
};

constexpr int WCHUNKS = 64;          // pixel chunks of the scalar weight-gradient kernels
constexpr int WCHUNKS_MAX = 1024;    // upper bound of the matrix-core and head chunk counts

template <class P>
static TrainBufs<P> train_layout(const no_net* net, const hz_problem* p, int B, void* base, size_t cap,
                                 bool recompute) {
    using T = typename P::T;
    TrainBufs<P> t;
    int Hp, Wp;
    net_padded_dims(net, p, &Hp, &Wp);
    Carver c(base, cap);
    // forward activations: carve with the same rules as fwd_layout, then continue after them
    t.f = fwd_layout<P>(net, Hp, Wp, B, base, cap, true, recompute);
    c.off = t.f.total;
    const int lv = net->a.levels;
    t.gA.resize(lv);
    t.gB.resize(lv);
    t.gU.resize(lv);
    t.gP.resize(lv);
    // gA, gU and gP live within one level's backward step (written in full, then read): one
    // scratch each for all levels; gB carries gradients from level to level
    size_t ga = 0, gp = 0;
    for (int l = 0; l < lv; ++l) {
        const size_t px = (size_t)B * (Hp >> l) * (Wp >> l);
        ga = std::max(ga, px * round16(net->a.base << l));
        if (l > 0) gp = std::max(gp, px * round16(net->a.base << (l - 1)));
    }
    T* gas = c.take<T>(ga);
    T* gus = lv > 1 ? c.take<T>(ga) : nullptr;
    T* gps = lv > 1 ? c.take<T>(gp) : nullptr;
    for (int l = 0; l < lv; ++l) {
        const size_t px = (size_t)B * (Hp >> l) * (Wp >> l);
        const int cs = round16(net->a.base << l);
        t.gA[l] = gas;
        t.gB[l] = c.take<T>(px * cs);
        t.gU[l] = l < lv - 1 ? gus : nullptr;
        t.gP[l] = l > 0 ? gps : nullptr;
    }
    const int64_t n = p->n;
    t.z = c.take<float2>((size_t)B * n);
    t.y = c.take<float2>((size_t)B * n);
    t.gz = c.take<float2>((size_t)B * n);
    Split sp = krylov_split(n);
    t.rpart = c.take<double2>((size_t)B * sp.nblk);
    t.ypart = c.take<double>((size_t)B * stencil_blocks(p));
    t.sc = c.take<double>(2 * (size_t)B);
    t.nr = c.take<double>(B);
    t.coef = c.take<float>(B);
    t.sprob = c.take<SampleProb>(B);
    size_t wmax = 0, bmax = 0;
    for (const Layer& ly : net->layers) {
        const int taps = ly.kind == L_CONV3 ? 9 : (ly.kind == L_CONVT2 ? 4 : 1);
        wmax = std::max(wmax, (size_t)WCHUNKS * taps * ly.cout_p * ly.cin_p);
        bmax = std::max(bmax, (size_t)WCHUNKS * (ly.cout_p + 2 * ly.cin_p + 2));
    }
    // the head's partials: one row of 2 cin_p + 2 per chunk
    const Layer& lh = net->layers.back();
    bmax = std::max(bmax, (size_t)WCHUNKS_MAX * (2 * lh.cin_p + 2));
    t.wpart = c.take<float>(wmax);
    t.wpartb = c.take<float>(bmax);
    t.wcap = wmax;
    t.bcap = bmax;
    t.total = c.off + 256;
    return t;
}

// ------------------------------------------------------------------ launch helpers

template <class P>
static int wgrad_conv3(const Layer& ly, const typename P::T* G, const typename P::T* x0, int c0,
                       const typename P::T* x1, int c1, int H, int W, int B, TrainBufs<P>& t, float* grad,
                       hipStream_t s) {
    const int ntiles = ((W + 15) / 16) * ((H + 7) / 8) * B;
    int nchunk;
    if constexpr (std::is_same<P, PolBF16>::value || std::is_same<P, PolF32>::value) {
        // matrix-core form: about 1024 blocks (512 in BF16, whose blocks prefetch their next tile),
        // as many chunks as the partial buffer holds
        const int ctiles = ((ly.cin_p + WG_CI - 1) / WG_CI) * ((ly.cout_p + WG_CO - 1) / WG_CO);
        const size_t per_chunk = (size_t)9 * ly.cout_p * ly.cin_p;
        const int nb = std::is_same<P, PolBF16>::value ? 512 : 1024;
        int want = std::min(512, std::max(1, (nb + ctiles - 1) / ctiles));
        want = (int)std::min<size_t>((size_t)want, t.wcap / per_chunk);
        want = std::min(want, (int)std::min<size_t>((size_t)WCHUNKS_MAX, t.bcap / (size_t)ly.cout_p));
        const int tpc = (ntiles + want - 1) / want;
        nchunk = (ntiles + tpc - 1) / tpc;
        dim3 grid((ly.cin_p + WG_CI - 1) / WG_CI, (ly.cout_p + WG_CO - 1) / WG_CO, nchunk);
        if constexpr (std::is_same<P, PolBF16>::value)
            hipLaunchKernelGGL(k_wgrad3_mfma, grid, dim3(TT), 0, s, G, ly.cout_p, x0, c0, x1, c1, H, W, ntiles, tpc,
                               t.wpart, t.wpartb);
        else
            hipLaunchKernelGGL(k_wgrad3_mfma_f32, grid, dim3(TT), 0, s, G, ly.cout_p, x0, c0, x1, c1, H, W, ntiles,
                               tpc, t.wpart, t.wpartb);
    } else {
        const int tpc = (ntiles + WCHUNKS - 1) / WCHUNKS;
        nchunk = (ntiles + tpc - 1) / tpc;
        dim3 grid((ly.cin_p + 15) / 16, ly.cout_p / 16, nchunk);
        hipLaunchKernelGGL(k_wgrad3<P>, grid, dim3(TT), 0, s, G, ly.cout_p, x0, c0, x1, c1, H, W, ntiles, tpc,
                           t.wpart, t.wpartb);
    }
    HZ_LAUNCH_CHECK();
    const int64_t nout = (int64_t)9 * ly.cin * ly.cout + ly.cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((nout + WR_OUT - 1) / WR_OUT)), dim3(WR_OUT * WR_GRP), 0, s,
                       t.wpart, t.wpartb, nchunk, ly, grad);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

template <class P>
static int wgrad_convT(const Layer& ly, const typename P::T* G, const typename P::T* x, int H, int W, int B,
                       TrainBufs<P>& t, float* grad, hipStream_t s) {
    int nchunk;
    if constexpr (std::is_same<P, PolBF16>::value) {
        const int ntiles = ((W + 15) / 16) * ((H + 7) / 8) * B;
        const int ctiles = ((ly.cin_p + WG_CI - 1) / WG_CI) * ((ly.cout_p + WG_CO - 1) / WG_CO);
        const size_t per_chunk = (size_t)4 * ly.cout_p * ly.cin_p;
        int want = std::min(512, std::max(1, (1024 + ctiles - 1) / ctiles));
        want = (int)std::min<size_t>((size_t)want, t.wcap / per_chunk);
        want = std::min(want, (int)std::min<size_t>((size_t)WCHUNKS_MAX, t.bcap / (size_t)ly.cout_p));
        const int tpc = (ntiles + want - 1) / want;
        nchunk = (ntiles + tpc - 1) / tpc;
        dim3 grid((ly.cin_p + WG_CI - 1) / WG_CI, (ly.cout_p + WG_CO - 1) / WG_CO, nchunk);
        hipLaunchKernelGGL(k_wgradT_mfma, grid, dim3(TT), 0, s, G, ly.cout_p, x, ly.cin_p, H, W, ntiles, tpc,
                           t.wpart, t.wpartb);
    } else {
        const int ntiles = ((W + 7) / 8) * ((H + 7) / 8) * B;
        const int tpc = (ntiles + WCHUNKS - 1) / WCHUNKS;
        nchunk = (ntiles + tpc - 1) / tpc;
        dim3 grid(ly.cin_p / 16, ly.cout_p / 16, nchunk);
        hipLaunchKernelGGL(k_wgradT<P>, grid, dim3(TT), 0, s, G, ly.cout_p, x, ly.cin_p, H, W, ntiles, tpc,
                           t.wpart, t.wpartb);
    }
    HZ_LAUNCH_CHECK();
    const int64_t nout = (int64_t)4 * ly.cin * ly.cout + ly.cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((nout + WR_OUT - 1) / WR_OUT)), dim3(WR_OUT * WR_GRP), 0, s,
                       t.wpart, t.wpartb, nchunk, ly, grad);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

// data gradient of a 3x3 layer: y0 (channels [0, split) or all) and y1 (rest), masks optional
template <class P>
static int dgrad_conv3(const no_net* net, const Layer& ly, const typename P::T* G, int H, int W, int B,
                       typename P::T* y0, typename P::T* y1, const typename P::T* mask0, const typename P::T* mask1,
                       hipStream_t s) {
    Conv3Out ex;
    ex.split = ly.cat_cp;
    ex.y1_ = y1;
    ex.mask0_ = mask0;
    ex.mask1_ = mask1;
    // output channels of the data gradient = stored input channels of the layer; BF16 layers whose
    // gradient has 1 or 2 chunks take the weight-stationary form (the same result bits)
    if (conv3_ws_dgrad_ok<P>(ly.cout_p, ly.cin_p, ly.cat_cp))
        return launch_conv3_ws_dgrad<P>(G, ly.cout_p, packed_wt<P>(net, ly), y0, ly.cin_p, H, W, B, ly.cat_cp, y1,
                                        mask0, mask1, s);
    return launch_conv3<P>(G, ly.cout_p, nullptr, 0, packed_wt<P>(net, ly), nullptr, y0, ly.cin_p, nullptr, H, W, B,
                           false, nullptr, s, ex);
}

template <class P>
static int dgrad_convT(const no_net* net, const Layer& ly, const typename P::T* G, const typename P::T* xmask,
                       typename P::T* gx, int H, int W, int B, hipStream_t s) {
    const int ck = std::min(P::CK, ly.cout_p);
    const int tn = ly.cin_p % 32 == 0 ? 32 : 16;
    dim3 grid((W + 63) / 64, H, (ly.cin_p / tn) * B);
    if (tn == 32)
        hipLaunchKernelGGL((k_convT2_dgrad<P, 32>), grid, dim3(TT), 0, s, G, ly.cout_p, packed_wt<P>(net, ly), xmask,
                           gx, ly.cin_p, H, W, ck);
    else
        hipLaunchKernelGGL((k_convT2_dgrad<P, 16>), grid, dim3(TT), 0, s, G, ly.cout_p, packed_wt<P>(net, ly), xmask,
                           gx, ly.cin_p, H, W, ck);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

// ------------------------------------------------------------------ per-sample batches

// ||r_b||^2 partials of every sample: block (q, b) covers [q per, (q + 1) per) of sample b.
__global__ __launch_bounds__(KT) void k_norm_batched(const float2* __restrict__ r, int64_t n, int64_t per,
                                                     double2* __restrict__ part, int nblk) {
    const int b = blockIdx.y;
    const int64_t p0 = (int64_t)blockIdx.x * per, p1 = min(n, p0 + per);
    norm_body(r + (int64_t)b * n, p0, p1, part + (int64_t)b * nblk + blockIdx.x);
}

// network input of every sample (sample b on grid row blockIdx.y), scale 1 / s_b = sc[2 b + 1]
template <class P>
__global__ void k_pack_batched(const float2* __restrict__ r, int64_t n, const double* __restrict__ sc,
                               const SampleProb* __restrict__ sp, int nxt, int nyt, int Hp, int Wp, int in_ch,
                               typename P::T* __restrict__ X) {
    const int b = blockIdx.y;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)Hp * Wp) return;
    const SampleProb& q = sp[b];
    pack_pixel<P, float2>(r + (int64_t)b * n, sc[2 * b + 1], q.cnd, q.sigx, q.sigy, nxt, nyt, Wp, in_ch,
                          X + (int64_t)b * Hp * Wp * 8, idx, nullptr, (float2*)nullptr);
}

// y_b = r_b - A_b z_b with one ||y_b||^2 partial per tile (sample b = blockIdx.z)
__global__ __launch_bounds__(ST_THREADS) void k_resid_batched(const float2* __restrict__ z, const float2* __restrict__ r,
                                                              float2* __restrict__ y, int64_t n,
                                                              const SampleProb* __restrict__ sp, int nxt, int nyt,
                                                              double* __restrict__ part) {
    const int b = blockIdx.z;
    const SampleProb& q = sp[b];
    const int64_t o = (int64_t)b * n;
    const int nst = gridDim.x * gridDim.y;
    stencil_tile<float, ST_RESID>(z + o, y + o, r + o, q.k2, q.fE, q.fW, q.fN, q.fS, q.dx, q.dy, 0, nxt, nyt,
                                  part + (int64_t)b * nst + blockIdx.y * gridDim.x + blockIdx.x, blockIdx.x * ST_TX,
                                  blockIdx.y * ST_TY);
}

// g_b = A_b^H y_b (sample b = blockIdx.z)
__global__ __launch_bounds__(ST_THREADS) void k_adjoint_batched(const float2* __restrict__ y, float2* __restrict__ g,
                                                                int64_t n, const SampleProb* __restrict__ sp, int nxt,
                                                                int nyt) {
    const int b = blockIdx.z;
    const SampleProb& q = sp[b];
    const int64_t o = (int64_t)b * n;
    stencil_tile<float, ST_PLAIN>(y + o, g + o, nullptr, q.k2, q.aE, q.aW, q.aN, q.aS, q.dx, q.dy, 1, nxt, nyt, nullptr,
                                  blockIdx.x * ST_TX, blockIdx.y * ST_TY);
}

// y_b = r_b - A_b z_b with ||y_b||^2 partials (stencil_blocks of them per sample) and, with grad,
// g_b = A_b^H y_b, for a batch on one grid: the finite-difference stencil in one launch per
// pass, or the Fourier-differentiation operator (Section 2.1) one sample at a time.
static int batch_resid_adjoint(int B, const hz_problem* const* probs, const float2* z, const float2* r, float2* y,
                               float2* gz, double* ypart, const SampleProb* sprob, bool grad, hipStream_t s) {
    const hz_problem* p0 = probs[0];
    const int64_t n = p0->n;
    if (is_spectral(p0)) {
        const int nst = stencil_blocks(p0);
        for (int b = 0; b < B; ++b)
            HZ_TRY(launch_spectral_resid32(probs[b], r + b * n, z + b * n, y + b * n, ypart + (int64_t)b * nst,
                                           nullptr, s));
        if (grad)
            for (int b = 0; b < B; ++b) HZ_TRY(launch_spectral(probs[b], false, true, y + b * n, gz + b * n, s, nullptr));
        return HZ_OK;
    }
    const dim3 g((p0->nxt + ST_TX - 1) / ST_TX, (p0->nyt + ST_TY - 1) / ST_TY, B);
    hipLaunchKernelGGL(k_resid_batched, g, dim3(ST_THREADS), 0, s, z, r, y, n, sprob, p0->nxt, p0->nyt, ypart);
    HZ_LAUNCH_CHECK();
    if (grad) {
        hipLaunchKernelGGL(k_adjoint_batched, g, dim3(ST_THREADS), 0, s, y, gz, n, sprob, p0->nxt, p0->nyt);
        HZ_LAUNCH_CHECK();
    }
    return HZ_OK;
}

// ------------------------------------------------------------------ loss + backward

template <class P>
static int loss_backward_impl(const no_net* net, int B, const hz_problem* const* probs, const float2* r, int squared,
                              bool recompute, float* loss, float* per_sample, float* grad, void* ws, size_t ws_bytes,
                              hipStream_t s) {
    using T = typename P::T;
    using Acc = typename P::Acc;
    const hz_problem* p0 = probs[0];
    TrainBufs<P> t = train_layout<P>(net, p0, B, ws, ws_bytes, recompute);
    if (t.total > ws_bytes) {
        set_error("no_loss_backward: workspace too small");
        return HZ_ERR_WORKSPACE;
    }
    int Hp, Wp;
    net_padded_dims(net, p0, &Hp, &Wp);
    const int64_t n = p0->n;
    const int lv = net->a.levels;
    const std::vector<Layer>& Ls = net->layers;
    Split sp = krylov_split(n);
    // the samples' problem pointers (one table, uploaded with the batch)
    {
        std::vector<SampleProb> hp(B);
        for (int b = 0; b < B; ++b) {
            const hz_problem* q = probs[b];
            hp[b] = SampleProb{q->k2f, q->cnd, q->sigx, q->sigy, q->fE_f, q->fW_f, q->fN_f, q->fS_f,
                               q->aE_f, q->aW_f, q->aN_f, q->aS_f, q->dx_f, q->dy_f};
        }
        HZ_HIP(hipMemcpyAsync(t.sprob, hp.data(), sizeof(SampleProb) * B, hipMemcpyHostToDevice, s));
    }
    // scales s_b and ||r_b||
    hipLaunchKernelGGL(k_norm_batched, dim3(sp.nblk, B), dim3(KT), 0, s, r, n, sp.per_block, t.rpart, sp.nblk);
    HZ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sample_scales, dim3(B), dim3(64), 0, s, t.rpart, sp.nblk, n, t.sc, t.nr);
    HZ_LAUNCH_CHECK();
    // pack every sample with its own velocity channel
    const unsigned gp = (unsigned)(((int64_t)Hp * Wp + 255) / 256);
    hipLaunchKernelGGL((k_pack_batched<P>), dim3(gp, B), dim3(256), 0, s, r, n, t.sc, t.sprob, p0->nxt, p0->nyt, Hp, Wp,
                       net->a.in_ch, (T*)t.f.X);
    HZ_LAUNCH_CHECK();
    // launch variants of the 3x3 layers at this batch (tuned on the first call of a size)
    HZ_TRY(net_autotune_bufs(net, Hp, Wp, B, t.f, prec_of<P>(), s));
    HZ_TRY(unet_body<P>(net, t.f, Hp, Wp, B, nullptr, s));
    const Layer& lh = Ls.back();
    const T* D0 = lv > 1 ? (const T*)t.f.D[0] : (const T*)t.f.E[0];
    {
        const int64_t tot = (int64_t)B * n;
        hipLaunchKernelGGL(k_head_batched<P>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, D0, lh.cin_p,
                           packed_w<P>(net, lh), packed_b<P>(net, lh), t.sc, p0->nxt, p0->nyt, Hp, Wp, B, t.z);
        HZ_LAUNCH_CHECK();
    }
    // y_b = r_b - A_b z_b with ||y_b||^2 partials, then A_b^H y_b
    const int nst = stencil_blocks(p0);
    HZ_TRY(batch_resid_adjoint(B, probs, t.z, r, t.y, t.gz, t.ypart, t.sprob, grad != nullptr, s));
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(1024), 0, s, t.ypart, nst, t.nr, B, squared, t.coef, loss, per_sample);
    HZ_LAUNCH_CHECK();
    if (!grad) return HZ_OK;  // loss only (validation): no reverse pass

    // ---- head
    {
        const int cs0 = lh.cin_p;
        const int64_t tot = (int64_t)B * Hp * Wp * (cs0 / (16 / (int)sizeof(T)));
        T* G0 = t.gB[0];
        hipLaunchKernelGGL(k_head_dgrad<P>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, t.gz, t.coef, t.sc,
                           D0, cs0, packed_w<P>(net, lh), p0->nxt, p0->nyt, Hp, Wp, B, G0);
        HZ_LAUNCH_CHECK();
        const int64_t np = (int64_t)B * Hp * Wp;
        const int64_t per = (np + WCHUNKS_MAX - 1) / WCHUNKS_MAX;
        const int nchunk = (int)((np + per - 1) / per);
        hipLaunchKernelGGL(k_head_wgrad<P>, dim3(nchunk), dim3(TT), 0, s, t.gz, t.coef, t.sc, D0, cs0, p0->nxt,
                           p0->nyt, Hp, Wp, B, per, t.wpartb);
        HZ_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_head_reduce, dim3((unsigned)((lh.cout * lh.cin + 2 + 3) / 4)), dim3(256), 0, s, t.wpartb,
                           nchunk, cs0, lh, grad);
        HZ_LAUNCH_CHECK();
    }
    // layer indices in the flat order
    std::vector<int> enc_a(lv), enc_b(lv), up(lv, -1), dec_a(lv, -1), dec_b(lv, -1);
    {
        int li = 0;
        for (int l = 0; l < lv; ++l) {
            enc_a[l] = li++;
            enc_b[l] = li++;
        }
        for (int l = lv - 2; l >= 0; --l) {
            up[l] = li++;
            dec_a[l] = li++;
            dec_b[l] = li++;
        }
    }
    // ---- decoder, level 0 upward; G of the current decoder-b layer is in gB[l]
    for (int l = 0; l <= lv - 2; ++l) {
        const int H = Hp >> l, W = Wp >> l;
        const Layer& lb = Ls[dec_b[l]];
        const Layer& la = Ls[dec_a[l]];
        const Layer& lu = Ls[up[l]];
        if (recompute) {
            // the level's upsampled tensor and first-convolution output, as the forward pass made them
            const T* Dn0 = l + 1 == lv - 1 ? (const T*)t.f.E[l + 1] : (const T*)t.f.D[l + 1];
            HZ_TRY(launch_convT2<P>(Dn0, lu.cin_p, packed_w<P>(net, lu), packed_b<P>(net, lu), (T*)t.f.U[l],
                                    lu.cout_p, H / 2, W / 2, B, nullptr, s));
            HZ_TRY(launch_conv3<P>((const T*)t.f.E[l], lu.cout_p, (const T*)t.f.U[l], lu.cout_p, packed_w<P>(net, la),
                                   packed_b<P>(net, la), (T*)t.f.T1d[l], la.cout_p, nullptr, H, W, B, true, nullptr,
                                   s, Conv3Out(), net_cfg(net, dec_a[l], H, W, B, prec_of<P>()),
                                   (Acc*)t.f.splitbuf));
        }
        const T* A1 = (const T*)t.f.T1d[l];
        HZ_TRY(wgrad_conv3<P>(lb, t.gB[l], A1, lb.cin_p, nullptr, 0, H, W, B, t, grad, s));
        HZ_TRY(dgrad_conv3<P>(net, lb, t.gB[l], H, W, B, t.gA[l], nullptr, A1, nullptr, s));
        HZ_TRY(wgrad_conv3<P>(la, t.gA[l], (const T*)t.f.E[l], la.cat_cp, (const T*)t.f.U[l], la.cin_p - la.cat_cp,
                              H, W, B, t, grad, s));
        // skip part (unmasked, completed by the pooling path) -> gB[l]; up part -> gU[l]
        HZ_TRY(dgrad_conv3<P>(net, la, t.gA[l], H, W, B, t.gB[l], t.gU[l], nullptr, nullptr, s));
        const T* Dn = l + 1 == lv - 1 ? (const T*)t.f.E[l + 1] : (const T*)t.f.D[l + 1];
        HZ_TRY(wgrad_convT<P>(lu, t.gU[l], Dn, H / 2, W / 2, B, t, grad, s));
        HZ_TRY(dgrad_convT<P>(net, lu, t.gU[l], Dn, t.gB[l + 1], H / 2, W / 2, B, s));
    }
    // ---- encoder, deepest level first; G(enc_lb) is in gB[l]
    for (int l = lv - 1; l >= 0; --l) {
        const int H = Hp >> l, W = Wp >> l;
        const Layer& lb = Ls[enc_b[l]];
        const Layer& la = Ls[enc_a[l]];
        const T* in = l == 0 ? (const T*)t.f.X : (const T*)t.f.P[l];
        if (recompute)   // the level's first-convolution output, as the forward pass made it
            HZ_TRY(launch_conv3<P>(in, la.cin_p, nullptr, 0, packed_w<P>(net, la), packed_b<P>(net, la),
                                   (T*)t.f.T1[l], la.cout_p, nullptr, H, W, B, true, nullptr, s, Conv3Out(),
                                   net_cfg(net, enc_a[l], H, W, B, prec_of<P>()), (Acc*)t.f.splitbuf));
        const T* A1 = (const T*)t.f.T1[l];
        HZ_TRY(wgrad_conv3<P>(lb, t.gB[l], A1, lb.cin_p, nullptr, 0, H, W, B, t, grad, s));
        HZ_TRY(dgrad_conv3<P>(net, lb, t.gB[l], H, W, B, t.gA[l], nullptr, A1, nullptr, s));
        HZ_TRY(wgrad_conv3<P>(la, t.gA[l], in, la.cin_p, nullptr, 0, H, W, B, t, grad, s));
        if (l > 0) {
            HZ_TRY(dgrad_conv3<P>(net, la, t.gA[l], H, W, B, t.gP[l], nullptr, nullptr, nullptr, s));
            const int Hu = Hp >> (l - 1), Wu = Wp >> (l - 1);
            const int c = Ls[enc_b[l - 1]].cout_p;
            const int64_t tot = (int64_t)B * Hu * Wu * c;
            const int64_t nv = tot / (16 / (int)sizeof(T));
            hipLaunchKernelGGL(k_pool_bwd<P>, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, t.gB[l - 1],
                               (const T*)t.gP[l], (const T*)t.f.E[l - 1], Hu, Wu, c, tot);
            HZ_LAUNCH_CHECK();
        }
    }
    return HZ_OK;
}

// ------------------------------------------------------------------ Table 2's network (FP32)
//
// Reverse mode of the 8x8 stride-2 layer set (Section 3.1, Table 2), in the paper's training
// precision (FP32). With s the pre-activation of a layer and g the gradient of its PReLU output:
//   PReLU:  gs = g (s > 0), alpha g (s <= 0); d alpha = sum_{s <= 0} s g; d b = sum gs;
//   weights: d W[m][n][tap] = sum over the coarse pixels (i, j) of coarse[i][j][m] times
//            fine[2i + a - 3][2j + e - 3][n] (tap = 8 a + e, fine values outside the grid are 0):
//            a strided convolution has coarse = gs, fine = its input (m = out, n = in channel), a
//            transposed one coarse = its input, fine = gs (m = in, n = out), matching the stored
//            [out][in][8][8] and [in][out][8][8] orders;
//   data:   the input gradient of a strided convolution is the transposed 8x8 form of gs with the
//            data-gradient pack, that of a transposed convolution the strided form (both through
//            k_conv8 with a linear epilogue: zero bias, slope 1);
//   the decoder's concat input splits its gradient into the skip part (added to the encoder
//   output's gradient) and the up part.
// All sums over pixels run in fixed orders (per-block partials, then the blocks in order).

constexpr int W8_CHUNKS = 16;    // pixel chunks of the 8x8 weight-gradient kernel
constexpr int PR_BLOCKS = 256;   // blocks of the PReLU backward (partial rows)

// In place: g <- gs = (g (+ g2)) * prelu'(s); part[blk][c] = sum gs (c < 32), part[blk][32] =
// sum_{s <= 0} s (g (+ g2)). 32 channels per pixel; thread (lane l of 8, channel c) strides over
// the block's pixels, then the 8 lanes are added in order.
__global__ __launch_bounds__(TT) void k_prelu8_bwd(float* __restrict__ g, const float* __restrict__ g2,
                                                   const float* __restrict__ spre, const float* __restrict__ bias,
                                                   int64_t npx, int64_t per, float* __restrict__ part) {
    const int c = threadIdx.x & 31, pl = threadIdx.x >> 5;
    const float alpha = bias[32];
    const int64_t p0 = (int64_t)blockIdx.x * per, p1 = min(npx, p0 + per);
    float db = 0.f, da = 0.f;
    for (int64_t p = p0 + pl; p < p1; p += 8) {
        const int64_t i = p * 32 + c;
        float v = g[i];
        if (g2) v += g2[i];
        const float sv = spre[i];
        const float gs = sv > 0.f ? v : alpha * v;
        if (!(sv > 0.f)) da += sv * v;
        g[i] = gs;
        db += gs;
    }
    __shared__ float rb[8][32], ra[TT];
    rb[pl][c] = db;
    ra[threadIdx.x] = da;
    __syncthreads();
    if (threadIdx.x < 32) {
        float t = 0.f;
        for (int l = 0; l < 8; ++l) t += rb[l][threadIdx.x];
        part[(int64_t)blockIdx.x * 33 + threadIdx.x] = t;
    }
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < TT; ++k) t += ra[k];
        part[(int64_t)blockIdx.x * 33 + 32] = t;
    }
}

// grad[b_off + c] = sum_blk part[blk][c] (c < 32), grad[a_off] = sum_blk part[blk][32], in block
// order.
__global__ void k_prelu8_reduce(const float* __restrict__ part, int nblk, int64_t b_off, int64_t a_off,
                                float* __restrict__ grad) {
    const int c = threadIdx.x;
    if (c > 32) return;
    float t = 0.f;
    for (int z = 0; z < nblk; ++z) t += part[(int64_t)z * 33 + c];
    if (c < 32) grad[b_off + c] = t;
    else grad[a_off] = t;
}

// Weight-gradient partials of one 8x8 layer on the matrix cores (v_mfma_f32_16x16x4_f32, 4 coarse
// pixels per instruction): block (tap, 16-row block of m, chunk z); its 4 wavefronts take the
// chunk's pixel quads round-robin, each for all n blocks, and are added in wavefront order.
// coarse: [B][Hc][Wc][cms] (channels m0 .. of it from column cmo), fine: [B][2Hc][2Wc][cns] (N
// channels used, N <= 32). part[z][(m * NP + n) * 64 + tap], NP = 32.
__global__ __launch_bounds__(TT) void k_wgrad8(const float* __restrict__ coarse, int cms, int cmo,
                                               const float* __restrict__ fine, int cns, int N, int Hc, int Wc, int B,
                                               int64_t per, float* __restrict__ part, int mrows) {
    const int tap = blockIdx.x, mb = blockIdx.y, z = blockIdx.z;
    const int a = tap >> 3, e = tap & 7;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int m = mb * 16 + col;   // A row of this lane
    const int64_t npx = (int64_t)B * Hc * Wc;
    const int64_t p0 = (int64_t)z * per, p1 = min(npx, p0 + per);
    const int Hf = 2 * Hc, Wf = 2 * Wc;
    f32x4_t acc[2] = {f32x4_t{0.f, 0.f, 0.f, 0.f}, f32x4_t{0.f, 0.f, 0.f, 0.f}};
    for (int64_t q = p0 + 4 * wv; q < p1; q += 16) {
        const int64_t p = q + kq;
        float av = 0.f, bv0 = 0.f, bv1 = 0.f;
        if (p < p1) {
            const int b = (int)(p / ((int64_t)Hc * Wc));
            const int r = (int)(p - (int64_t)b * Hc * Wc);
            const int i = r / Wc, j = r - (r / Wc) * Wc;
            av = coarse[p * cms + cmo + m];
            const int fy = 2 * i + a - 3, fx = 2 * j + e - 3;
            if (fy >= 0 && fy < Hf && fx >= 0 && fx < Wf) {
                const float* fr = fine + (((int64_t)b * Hf + fy) * Wf + fx) * cns;
                if (col < N) bv0 = fr[col];
                if (16 + col < N) bv1 = fr[16 + col];
            }
        }
        acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv1, acc[1], 0, 0, 0);
    }
    __shared__ f32x4_t red[4][2][64];
    red[wv][0][lane] = acc[0];
    red[wv][1][lane] = acc[1];
    __syncthreads();
    if (wv != 0) return;
    f32x4_t t0 = red[0][0][lane], t1 = red[0][1][lane];
    for (int w = 1; w < 4; ++w) {
        t0 += red[w][0][lane];
        t1 += red[w][1][lane];
    }
    // D layout: lane l holds rows 4 (l / 16) + r (m) of column l % 16 (n)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int mm = mb * 16 + 4 * kq + r;
        if (mm >= mrows) continue;
        float* dst = part + (int64_t)z * mrows * 32 * 64;
        if (col < N) dst[((int64_t)mm * 32 + col) * 64 + tap] = t0[r];
        if (16 + col < N) dst[((int64_t)mm * 32 + 16 + col) * 64 + tap] = t1[r];
    }
}

// grad[w_off + (m * Nl + n) * 64 + tap] = sum_z part[z][(m * 32 + n) * 64 + tap] (m < Ml, n < Nl),
// chunks in order.
__global__ void k_wgrad8_reduce(const float* __restrict__ part, int nchunk, int mrows, int Ml, int Nl, int64_t w_off,
                                float* __restrict__ grad) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)Ml * Nl * 64) return;
    const int tap = (int)(t % 64);
    const int n = (int)((t / 64) % Nl);
    const int m = (int)(t / (64 * Nl));
    const int64_t slot = ((int64_t)m * 32 + n) * 64 + tap;
    float a = 0.f;
    for (int z = 0; z < nchunk; ++z) a += part[(int64_t)z * mrows * 32 * 64 + slot];
    grad[w_off + t] = a;
}

// G(U0)[p][c] = g0 Wh[0][c] + g1 Wh[1][c] (the PReLU of the last up layer is handled by its own
// backward step).
__global__ void k_head8_dgrad(const float2* __restrict__ gz, const float* __restrict__ coef,
                              const double* __restrict__ sc, const float* __restrict__ wh, int nxt, int nyt, int Hp,
                              int Wp, int B, float* __restrict__ G) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = (int64_t)Hp * Wp;
    if (idx >= np * B * 32) return;
    const int c = (int)(idx % 32);
    const int64_t pp = idx / 32;
    const int b = (int)(pp / np);
    const int64_t q = pp - (int64_t)b * np;
    const float2 g = head_grad(gz, coef, sc, b, (int)(q / Wp), (int)(q % Wp), nxt, nyt);
    G[idx] = g.x * wh[c] + g.y * wh[32 + c];
}

// linear epilogue of the data-gradient launches: zero bias, PReLU slope 1
__global__ void k_linear_bias(float* b) {
    if (threadIdx.x < 33) b[threadIdx.x] = threadIdx.x == 32 ? 1.f : 0.f;
}

struct Train8Bufs {
    FwdBufs f;                      // X, E[1..L], U[0..L-1] (the forward's activations)
    std::vector<float*> sE, sU;     // pre-activations
    std::vector<float*> gE, gU;     // activation gradients
    float* tmp;                     // data gradient of a strided convolution (finest level size)
    float2 *z, *y, *gz;
    double2* rpart;
    double* ypart;
    double *sc, *nr;
    float* coef;
    SampleProb* sprob;
    float *wpart, *ppart, *lin;
    size_t total;
};

static Train8Bufs train8_layout(const no_net* net, const hz_problem* p, int B, void* base, size_t cap) {
    Train8Bufs t;
    int Hp, Wp;
    net_padded_dims(net, p, &Hp, &Wp);
    t.f = fwd_layout<PolF32>(net, Hp, Wp, B, base, cap);
    Carver c(base, cap);
    c.off = t.f.total;
    const int lv = net->a.levels;
    t.sE.assign(lv + 1, nullptr);
    t.gE.assign(lv + 1, nullptr);
    t.sU.assign(lv, nullptr);
    t.gU.assign(lv, nullptr);
    for (int l = 1; l <= lv; ++l) {
        const size_t px = (size_t)B * (Hp >> l) * (Wp >> l);
        t.sE[l] = c.take<float>(px * 32);
        t.gE[l] = c.take<float>(px * 32);
    }
    for (int l = 0; l < lv; ++l) {
        const size_t px = (size_t)B * (Hp >> l) * (Wp >> l);
        t.sU[l] = c.take<float>(px * 32);
        t.gU[l] = c.take<float>(px * 32);
    }
    t.tmp = c.take<float>((size_t)B * (Hp >> 1) * (Wp >> 1) * 32);
    const int64_t n = p->n;
    t.z = c.take<float2>((size_t)B * n);
    t.y = c.take<float2>((size_t)B * n);
    t.gz = c.take<float2>((size_t)B * n);
    Split sp = krylov_split(n);
    t.rpart = c.take<double2>((size_t)B * sp.nblk);
    t.ypart = c.take<double>((size_t)B * stencil_blocks(p));
    t.sc = c.take<double>(2 * (size_t)B);
    t.nr = c.take<double>(B);
    t.coef = c.take<float>(B);
    t.sprob = c.take<SampleProb>(B);
    t.wpart = c.take<float>((size_t)W8_CHUNKS * 64 * 32 * 64);
    const Layer& lh = net->layers.back();
    t.ppart = c.take<float>(std::max<size_t>((size_t)PR_BLOCKS * 33, (size_t)WCHUNKS_MAX * (2 * lh.cin_p + 2)));
    t.lin = c.take<float>(64);
    t.total = c.off + 256;
    return t;
}

// d W of one 8x8 layer into the flat gradient; coarse given as up to two channel parts of 32
static int wgrad8(const Layer& ly, const float* c0p, const float* c1p, int cms0, int cms1, const float* fine, int cns,
                  int N, int Hc, int Wc, int B, Train8Bufs& t, float* grad, int Ml, int Nl, hipStream_t s) {
    const int64_t npx = (int64_t)B * Hc * Wc;
    const int64_t per = ((npx + W8_CHUNKS - 1) / W8_CHUNKS + 15) / 16 * 16;
    const int nchunk = (int)((npx + per - 1) / per);
    const int mrows = Ml > 32 ? 64 : 32;
    // first part: rows [0, 32) from c0p; second (concat): rows [32, 64) from c1p
    hipLaunchKernelGGL(k_wgrad8, dim3(64, 2, nchunk), dim3(TT), 0, s, c0p, cms0, 0, fine, cns, N, Hc, Wc, B, per,
                       t.wpart, mrows);
    HZ_LAUNCH_CHECK();
    if (c1p) {
        hipLaunchKernelGGL(k_wgrad8, dim3(64, 2, nchunk), dim3(TT), 0, s, c1p, cms1, 0, fine, cns, N, Hc, Wc, B, per,
                           t.wpart + (int64_t)32 * 32 * 64, mrows);
        HZ_LAUNCH_CHECK();
    }
    const int64_t nout = (int64_t)Ml * Nl * 64;
    hipLaunchKernelGGL(k_wgrad8_reduce, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, t.wpart, nchunk, mrows,
                       Ml, Nl, ly.w_off, grad);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

static int prelu8_bwd(const Layer& ly, const no_net* net, float* g, const float* g2, const float* spre, int64_t npx,
                      Train8Bufs& t, float* grad, hipStream_t s) {
    const int64_t per = (npx + PR_BLOCKS - 1) / PR_BLOCKS;
    const int nblk = (int)((npx + per - 1) / per);
    hipLaunchKernelGGL(k_prelu8_bwd, dim3(nblk), dim3(TT), 0, s, g, g2, spre, packed_b<PolF32>(net, ly), npx, per,
                       t.ppart);
    HZ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_prelu8_reduce, dim3(1), dim3(64), 0, s, t.ppart, nblk, ly.b_off, ly.a_off, grad);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

size_t train8_ws_bytes(const no_net* net, const hz_problem* p, int B) {
    return train8_layout(net, p, B, nullptr, 0).total;
}

int loss_backward8(const no_net* net, int B, const hz_problem* const* probs, const float2* r, int squared,
                   float* loss, float* per_sample, float* grad, void* ws, size_t ws_bytes, hipStream_t s) {
    using P = PolF32;
    const hz_problem* p0 = probs[0];
    Train8Bufs t = train8_layout(net, p0, B, ws, ws_bytes);
    if (t.total > ws_bytes) {
        set_error("no_loss_backward: workspace too small");
        return HZ_ERR_WORKSPACE;
    }
    int Hp, Wp;
    net_padded_dims(net, p0, &Hp, &Wp);
    const int64_t n = p0->n;
    const int lv = net->a.levels;
    const std::vector<Layer>& Ls = net->layers;
    Split sp = krylov_split(n);
    {
        std::vector<SampleProb> hp(B);
        for (int b = 0; b < B; ++b) {
            const hz_problem* q = probs[b];
            hp[b] = SampleProb{q->k2f, q->cnd, q->sigx, q->sigy, q->fE_f, q->fW_f, q->fN_f, q->fS_f,
                               q->aE_f, q->aW_f, q->aN_f, q->aS_f, q->dx_f, q->dy_f};
        }
        HZ_HIP(hipMemcpyAsync(t.sprob, hp.data(), sizeof(SampleProb) * B, hipMemcpyHostToDevice, s));
    }
    hipLaunchKernelGGL(k_norm_batched, dim3(sp.nblk, B), dim3(KT), 0, s, r, n, sp.per_block, t.rpart, sp.nblk);
    HZ_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sample_scales, dim3(B), dim3(64), 0, s, t.rpart, sp.nblk, n, t.sc, t.nr);
    HZ_LAUNCH_CHECK();
    const unsigned gp = (unsigned)(((int64_t)Hp * Wp + 255) / 256);
    hipLaunchKernelGGL((k_pack_batched<P>), dim3(gp, B), dim3(256), 0, s, r, n, t.sc, t.sprob, p0->nxt, p0->nyt, Hp, Wp,
                       net->a.in_ch, (float*)t.f.X);
    HZ_LAUNCH_CHECK();
    // forward, keeping the pre-activations
    std::vector<int> dn(lv + 1), upl(lv);
    {
        int li = 0;
        for (int l = 1; l <= lv; ++l) dn[l] = li++;
        upl[lv - 1] = li++;
        for (int l = lv - 2; l >= 0; --l) upl[l] = li++;
    }
    const float* in = (const float*)t.f.X;
    for (int l = 1; l <= lv; ++l) {
        const Layer& ly = Ls[dn[l]];
        HZ_TRY(launch_conv8<P>(false, in, nullptr, ly.cin_p, 0, packed_w<P>(net, ly), packed_b<P>(net, ly),
                               (float*)t.f.E[l], 32, Hp >> (l - 1), Wp >> (l - 1), B, nullptr, s, t.sE[l]));
        in = (const float*)t.f.E[l];
    }
    {
        const Layer& ly = Ls[upl[lv - 1]];
        HZ_TRY(launch_conv8<P>(true, (const float*)t.f.E[lv], nullptr, ly.cin_p, 0, packed_w<P>(net, ly),
                               packed_b<P>(net, ly), (float*)t.f.U[lv - 1], 32, Hp >> lv, Wp >> lv, B, nullptr, s,
                               t.sU[lv - 1]));
    }
    for (int l = lv - 2; l >= 0; --l) {
        const Layer& ly = Ls[upl[l]];
        HZ_TRY(launch_conv8<P>(true, (const float*)t.f.E[l + 1], (const float*)t.f.U[l + 1], ly.cin_p, ly.cat_cp,
                               packed_w<P>(net, ly), packed_b<P>(net, ly), (float*)t.f.U[l], 32, Hp >> (l + 1),
                               Wp >> (l + 1), B, nullptr, s, t.sU[l]));
    }
    const Layer& lh = Ls.back();
    const float* U0 = (const float*)t.f.U[0];
    {
        const int64_t tot = (int64_t)B * n;
        hipLaunchKernelGGL(k_head_batched<P>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, U0, lh.cin_p,
                           packed_w<P>(net, lh), packed_b<P>(net, lh), t.sc, p0->nxt, p0->nyt, Hp, Wp, B, t.z);
        HZ_LAUNCH_CHECK();
    }
    const int nst = stencil_blocks(p0);
    HZ_TRY(batch_resid_adjoint(B, probs, t.z, r, t.y, t.gz, t.ypart, t.sprob, grad != nullptr, s));
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(1024), 0, s, t.ypart, nst, t.nr, B, squared, t.coef, loss, per_sample);
    HZ_LAUNCH_CHECK();
    if (!grad) return HZ_OK;

    // ---- head
    {
        const int64_t tot = (int64_t)B * Hp * Wp * 32;
        hipLaunchKernelGGL(k_head8_dgrad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, t.gz, t.coef, t.sc,
                           packed_w<P>(net, lh), p0->nxt, p0->nyt, Hp, Wp, B, t.gU[0]);
        HZ_LAUNCH_CHECK();
        const int64_t np = (int64_t)B * Hp * Wp;
        const int64_t per = (np + WCHUNKS_MAX - 1) / WCHUNKS_MAX;
        const int nchunk = (int)((np + per - 1) / per);
        hipLaunchKernelGGL(k_head_wgrad<P>, dim3(nchunk), dim3(TT), 0, s, t.gz, t.coef, t.sc, U0, lh.cin_p, p0->nxt,
                           p0->nyt, Hp, Wp, B, per, t.ppart);
        HZ_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_head_reduce, dim3((unsigned)((lh.cout * lh.cin + 2 + 3) / 4)), dim3(256), 0, s, t.ppart,
                           nchunk, lh.cin_p, lh, grad);
        HZ_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_linear_bias, dim3(1), dim3(64), 0, s, t.lin);
    HZ_LAUNCH_CHECK();
    // ---- decoder, finest level first: gU[l] holds the gradient of U_l
    for (int l = 0; l < lv; ++l) {
        const Layer& ly = Ls[upl[l]];
        const int Hc = Hp >> (l + 1), Wc = Wp >> (l + 1);   // the layer's input size
        const int64_t npx = (int64_t)B * (Hp >> l) * (Wp >> l);
        HZ_TRY(prelu8_bwd(ly, net, t.gU[l], nullptr, t.sU[l], npx, t, grad, s));
        const float* gs = t.gU[l];
        const bool cat = l < lv - 1;
        // d W[c][o][tap]: coarse = the input (E_{l+1} | U_{l+1}), fine = gs
        HZ_TRY(wgrad8(ly, (const float*)t.f.E[l + 1], cat ? (const float*)t.f.U[l + 1] : nullptr, 32, 32, gs, 32, 32,
                      Hc, Wc, B, t, grad, ly.cin, ly.cout, s));
        // input gradient: the strided form of gs with the data-gradient pack [tap][cin_p][32]
        const float* wt = packed_wt<P>(net, ly);
        HZ_TRY(launch_conv8<P>(false, gs, nullptr, 32, 0, wt, t.lin, t.gE[l + 1], 32, Hp >> l, Wp >> l, B, nullptr, s,
                               nullptr, ly.cin_p));
        if (cat)
            HZ_TRY(launch_conv8<P>(false, gs, nullptr, 32, 0, wt + 32 * 32, t.lin, t.gU[l + 1], 32, Hp >> l, Wp >> l,
                                   B, nullptr, s, nullptr, ly.cin_p));
    }
    // ---- encoder, deepest first: the gradient of E_l is gE[l] (+ the strided layer above's data
    // gradient in tmp, for l < L)
    for (int l = lv; l >= 1; --l) {
        const Layer& ly = Ls[dn[l]];
        const int64_t npx = (int64_t)B * (Hp >> l) * (Wp >> l);
        HZ_TRY(prelu8_bwd(ly, net, t.gE[l], l < lv ? t.tmp : nullptr, t.sE[l], npx, t, grad, s));
        const float* gs = t.gE[l];
        const float* xin = l == 1 ? (const float*)t.f.X : (const float*)t.f.E[l - 1];
        const int cs_in = l == 1 ? 8 : 32;
        // d W[o][c][tap]: coarse = gs, fine = the input
        HZ_TRY(wgrad8(ly, gs, nullptr, 32, 0, xin, cs_in, cs_in, Hp >> l, Wp >> l, B, t, grad, ly.cout, ly.cin, s));
        if (l > 1)   // input gradient: the transposed form of gs with the data-gradient pack [tap][32][32]
            HZ_TRY(launch_conv8<P>(true, gs, nullptr, 32, 0, packed_wt<P>(net, ly), t.lin, t.tmp, 32, Hp >> l,
                                   Wp >> l, B, nullptr, s, nullptr, 32));
    }
    return HZ_OK;
}

// ------------------------------------------------------------------ Adam

__global__ void k_sqnorm_part(const float* __restrict__ g, int64_t n, double* __restrict__ part) {
    double a = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a += (double)g[i] * g[i];
    __shared__ double red[4];
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, const double* __restrict__ part, int nparts, int step,
                       float lr, float b1, float b2, float eps, float clip) {
    __shared__ double scale;
    if (threadIdx.x == 0) {
        double a = 0;
        for (int q = 0; q < nparts; ++q) a += part[q];
        const double nrm = sqrt(a);
        scale = (clip > 0 && nrm > clip) ? clip / nrm : 1.0;
    }
    __syncthreads();
    const float sc = (float)scale;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i] * sc;
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

constexpr int ADAM_BLOCKS = 512;

}  // namespace hz

using namespace hz;

extern "C" size_t no_train_workspace_size(const no_net* net, const hz_problem* p, int batch, no_prec prec,
                                          int recompute) {
    clear_error();
    if (!net || !p || batch < 1) return 0;
    if (net->a.kind == NO_ARCH_PAPER8) return prec == NO_FP32 && !recompute ? train8_ws_bytes(net, p, batch) : 0;
    if (prec == NO_BF16) return train_layout<PolBF16>(net, p, batch, nullptr, 0, recompute != 0).total;
    if (prec == NO_FP32) return train_layout<PolF32>(net, p, batch, nullptr, 0, recompute != 0).total;
    return 0;
}

extern "C" int no_loss_backward(const no_net* net, int batch, const hz_problem* const* problems, const void* r,
                                int squared, int recompute, no_prec prec, float* loss, float* per_sample, float* grad,
                                void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    HZ_CHECK_ARG(net && problems && r && loss && ws, "no_loss_backward: NULL argument");
    HZ_CHECK_ARG(net->a.kind == NO_ARCH_UNET3 || (prec == NO_FP32 && !recompute),
                 "no_loss_backward: Table 2's network trains in FP32 without activation checkpointing");
    HZ_CHECK_ARG(batch >= 1 && batch <= 1024, "no_loss_backward: batch must be in [1, 1024]");
    HZ_CHECK_ARG(prec == NO_BF16 || prec == NO_FP32, "no_loss_backward: precision must be NO_BF16 or NO_FP32");
    for (int b = 0; b < batch; ++b) {
        HZ_CHECK_ARG(problems[b], "no_loss_backward: NULL problem");
        HZ_CHECK_ARG(problems[b]->nxt == problems[0]->nxt && problems[b]->nyt == problems[0]->nyt &&
                         problems[b]->g.npml == problems[0]->g.npml,
                     "no_loss_backward: every problem of a batch must have the same grid and PML");
        HZ_CHECK_ARG(is_spectral(problems[b]) == is_spectral(problems[0]),
                     "no_loss_backward: every problem of a batch must have the same discretization");
    }
    hipStream_t s = (hipStream_t)stream;
    if (net->a.kind == NO_ARCH_PAPER8)
        return loss_backward8(net, batch, problems, (const float2*)r, squared, loss, per_sample, grad, ws, ws_bytes, s);
    if (prec == NO_BF16)
        return loss_backward_impl<PolBF16>(net, batch, problems, (const float2*)r, squared, recompute != 0, loss,
                                           per_sample, grad, ws, ws_bytes, s);
    return loss_backward_impl<PolF32>(net, batch, problems, (const float2*)r, squared, recompute != 0, loss,
                                      per_sample, grad, ws, ws_bytes, s);
}

extern "C" size_t no_adam_workspace_size(const no_net* net) {
    (void)net;
    return ADAM_BLOCKS * sizeof(double) + 256;
}

extern "C" int no_adam_step(no_net* net, float* theta, float* m, float* v, const float* grad, int step, float lr,
                            float b1, float b2, float eps, float clip, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    HZ_CHECK_ARG(net && theta && m && v && grad && ws, "no_adam_step: NULL argument");
    HZ_CHECK_ARG(step >= 1 && lr > 0 && b1 >= 0 && b1 < 1 && b2 >= 0 && b2 < 1 && eps > 0,
                 "no_adam_step: bad hyper-parameters");
    if (ws_bytes < no_adam_workspace_size(net)) {
        set_error("no_adam_step: workspace too small");
        return HZ_ERR_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    double* part = (double*)ws;
    hipLaunchKernelGGL(k_sqnorm_part, dim3(ADAM_BLOCKS), dim3(256), 0, s, grad, net->nparam, part);
    hipLaunchKernelGGL(k_adam, dim3(ADAM_BLOCKS), dim3(256), 0, s, theta, m, v, grad, net->nparam, part, ADAM_BLOCKS,
                       step, lr, b1, b2, eps, clip);
    HZ_LAUNCH_CHECK();
    return no_net_set_weights(net, theta, stream);
}
