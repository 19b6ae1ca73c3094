// Device body of the five-point complex Helmholtz stencil (shared by the single-system and
// the ragged-batch kernels).
#pragma once

#include "common.h"

namespace hz {

enum StencilMode { ST_PLAIN = 0, ST_RESID = 1 };

constexpr int ST_TX = 64, ST_TY = 16, ST_THREADS = 256;

// One 64 x 16 output tile per block of 256 threads; the (16+2) x (64+2) input
// tile with its one-node halo is staged in LDS (zero outside the grid), then
// each thread produces 4 outputs of one column from LDS.
template <typename T, int MODE>
__device__ __forceinline__ void stencil_tile(
    const cplx_t<T>* __restrict__ u, cplx_t<T>* __restrict__ y, const cplx_t<T>* __restrict__ b,
    const T* __restrict__ k2, const cplx_t<T>* __restrict__ cE, const cplx_t<T>* __restrict__ cW,
    const cplx_t<T>* __restrict__ cN, const cplx_t<T>* __restrict__ cS,
    const cplx_t<T>* __restrict__ dx, const cplx_t<T>* __restrict__ dy, int conj_diag, int nx, int ny,
    double* __restrict__ part_slot, int i0, int j0) {
    using C = cplx_t<T>;
    __shared__ C tile[ST_TY + 2][ST_TX + 2];
    for (int t = threadIdx.x; t < (ST_TY + 2) * (ST_TX + 2); t += ST_THREADS) {
        int ly = t / (ST_TX + 2), lx = t - ly * (ST_TX + 2);
        int gi = i0 + lx - 1, gj = j0 + ly - 1;
        C v{0, 0};
        if (gi >= 0 && gi < nx && gj >= 0 && gj < ny) v = u[(int64_t)gj * nx + gi];
        tile[ly][lx] = v;
    }
    __syncthreads();
    const int lx = threadIdx.x % ST_TX, ly0 = threadIdx.x / ST_TX;
    const int gi = i0 + lx;
    double nacc = 0.0;
    if (gi < nx) {
        const C e = cE[gi], w = cW[gi], dxi = dx[gi];
        for (int r = ly0; r < ST_TY; r += ST_THREADS / ST_TX) {
            const int gj = j0 + r;
            if (gj >= ny) break;
            const int64_t idx = (int64_t)gj * nx + gi;
            C d = C{k2[idx] - dxi.x - dy[gj].x, -dxi.y - dy[gj].y};
            if (conj_diag) d.y = -d.y;
            C acc = cmul(d, tile[r + 1][lx + 1]);
            acc = cadd(acc, cmul(e, tile[r + 1][lx + 2]));
            acc = cadd(acc, cmul(w, tile[r + 1][lx]));
            acc = cadd(acc, cmul(cN[gj], tile[r + 2][lx + 1]));
            acc = cadd(acc, cmul(cS[gj], tile[r][lx + 1]));
            if (MODE == ST_RESID) {
                C bb = b[idx];
                acc = C{bb.x - acc.x, bb.y - acc.y};
                nacc += (double)acc.x * acc.x + (double)acc.y * acc.y;
            }
            y[idx] = acc;
        }
    }
    if (MODE == ST_RESID) {
        __shared__ double red[ST_THREADS / 64];
        nacc = wave_sum(nacc);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nacc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0;
            for (int q = 0; q < ST_THREADS / 64; ++q) s += red[q];
            *part_slot = s;
        }
    }
}

// FP32 operator on a 64 x 32 output tile (nx even, 16-byte aligned u and y): the (32 + 2) x 64
// interior of the input tile is staged in LDS with 16-byte loads (two points each), the two halo
// columns with 8-byte loads; thread (c, r) computes the point pair (2c, 2c + 1) of rows r, r + 8,
// r + 16, r + 24 and stores each pair with one 16-byte store. Same term order as stencil_tile.
constexpr int SW_TX = 64, SW_TY = 32;
__device__ __forceinline__ void stencil_tile_wide(const float2* __restrict__ u, float2* __restrict__ y,
                                                  const float* __restrict__ k2, const float2* __restrict__ cE,
                                                  const float2* __restrict__ cW, const float2* __restrict__ cN,
                                                  const float2* __restrict__ cS, const float2* __restrict__ dx,
                                                  const float2* __restrict__ dy, int conj_diag, int nx, int ny,
                                                  int i0, int j0) {
    using C = float2;
    __shared__ __attribute__((aligned(16))) float4 mid[SW_TY + 2][SW_TX / 2];   // columns i0 .. i0 + 63
    __shared__ C hal[SW_TY + 2][2];                                              // columns i0 - 1, i0 + 64
    const int hq = nx >> 1;
    const float4* __restrict__ u4 = (const float4*)u;
    for (int t = threadIdx.x; t < (SW_TY + 2) * (SW_TX / 2); t += 256) {
        const int ly = t / (SW_TX / 2), lc = t - ly * (SW_TX / 2);
        const int gj = j0 + ly - 1, gi = i0 + 2 * lc;
        float4 v{0.f, 0.f, 0.f, 0.f};
        if (gj >= 0 && gj < ny && gi < nx) v = u4[(int64_t)gj * hq + (gi >> 1)];
        mid[ly][lc] = v;
    }
    for (int t = threadIdx.x; t < (SW_TY + 2) * 2; t += 256) {
        const int ly = t >> 1, side = t & 1;
        const int gj = j0 + ly - 1, gi = side ? i0 + SW_TX : i0 - 1;
        C v{0.f, 0.f};
        if (gj >= 0 && gj < ny && gi >= 0 && gi < nx) v = u[(int64_t)gj * nx + gi];
        hal[ly][side] = v;
    }
    __syncthreads();
    const int c = threadIdx.x & 31, r0 = threadIdx.x >> 5;
    const int gi = i0 + 2 * c;
    if (gi >= nx) return;
    const C e0 = cE[gi], e1 = cE[gi + 1], w0 = cW[gi], w1 = cW[gi + 1], x0 = dx[gi], x1 = dx[gi + 1];
#pragma unroll
    for (int k = 0; k < SW_TY / 8; ++k) {
        const int r = r0 + 8 * k, gj = j0 + r;
        if (gj >= ny) break;
        const float4 cc = mid[r + 1][c], nn = mid[r + 2][c], ss = mid[r][c];
        const C uw = c > 0 ? C{mid[r + 1][c - 1].z, mid[r + 1][c - 1].w} : hal[r + 1][0];
        const C ue = c < SW_TX / 2 - 1 ? C{mid[r + 1][c + 1].x, mid[r + 1][c + 1].y} : hal[r + 1][1];
        const int64_t p = (int64_t)gj * nx + gi;
        const float2 kk = *(const float2*)(k2 + p);
        const C dyj = dy[gj], nj = cN[gj], sj = cS[gj];
        const C u0{cc.x, cc.y}, u1{cc.z, cc.w};
        C d0 = C{kk.x - x0.x - dyj.x, -x0.y - dyj.y};
        C d1 = C{kk.y - x1.x - dyj.x, -x1.y - dyj.y};
        if (conj_diag) {
            d0.y = -d0.y;
            d1.y = -d1.y;
        }
        C a0 = cmul(d0, u0);
        a0 = cadd(a0, cmul(e0, u1));
        a0 = cadd(a0, cmul(w0, uw));
        a0 = cadd(a0, cmul(nj, C{nn.x, nn.y}));
        a0 = cadd(a0, cmul(sj, C{ss.x, ss.y}));
        C a1 = cmul(d1, u1);
        a1 = cadd(a1, cmul(e1, ue));
        a1 = cadd(a1, cmul(w1, u0));
        a1 = cadd(a1, cmul(nj, C{nn.z, nn.w}));
        a1 = cadd(a1, cmul(sj, C{ss.z, ss.w}));
        // streaming (non-temporal) store: this kernel never reads its output
        typedef float f4v __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(f4v{a0.x, a0.y, a1.x, a1.y}, (f4v*)(y + p));
    }
}

// The same operator for the two adjacent points (p, p + 1) = (gi, gi + 1) of one row, gi even,
// nx even, u / y 16-byte aligned: the centre, north and south pairs are 16-byte loads, the west
// and east neighbours 8-byte loads (zero outside the grid), the result one 16-byte store. Same
// term order as stencil_tile.
__device__ __forceinline__ float4 stencil_pair_value(const float2* __restrict__ u,
                                                     const float* __restrict__ k2, const float2* __restrict__ cE,
                                                     const float2* __restrict__ cW, const float2* __restrict__ cN,
                                                     const float2* __restrict__ cS, const float2* __restrict__ dx,
                                                     const float2* __restrict__ dy, int conj_diag, int nx, int ny,
                                                     int64_t p) {
    using C = float2;
    const int gj = (int)(p / nx), gi = (int)(p - (int64_t)gj * nx);
    const int64_t q = p >> 1, hq = nx >> 1;
    const float4* __restrict__ u4 = (const float4*)u;
    const float4 c = u4[q];
    const float4 zero4{0.f, 0.f, 0.f, 0.f};
    const float4 nn = gj + 1 < ny ? u4[q + hq] : zero4;
    const float4 ss = gj > 0 ? u4[q - hq] : zero4;
    const C uw = gi > 0 ? u[p - 1] : C{0.f, 0.f};
    const C ue = gi + 2 < nx ? u[p + 2] : C{0.f, 0.f};
    const float2 kk = ((const float2*)k2)[q];
    const C dyj = dy[gj], nj = cN[gj], sj = cS[gj];
    const C u0{c.x, c.y}, u1{c.z, c.w};
    C d0 = C{kk.x - dx[gi].x - dyj.x, -dx[gi].y - dyj.y};
    C d1 = C{kk.y - dx[gi + 1].x - dyj.x, -dx[gi + 1].y - dyj.y};
    if (conj_diag) {
        d0.y = -d0.y;
        d1.y = -d1.y;
    }
    C a0 = cmul(d0, u0);
    a0 = cadd(a0, cmul(cE[gi], u1));
    a0 = cadd(a0, cmul(cW[gi], uw));
    a0 = cadd(a0, cmul(nj, C{nn.x, nn.y}));
    a0 = cadd(a0, cmul(sj, C{ss.x, ss.y}));
    C a1 = cmul(d1, u1);
    a1 = cadd(a1, cmul(cE[gi + 1], ue));
    a1 = cadd(a1, cmul(cW[gi + 1], u0));
    a1 = cadd(a1, cmul(nj, C{nn.z, nn.w}));
    a1 = cadd(a1, cmul(sj, C{ss.z, ss.w}));
    return float4{a0.x, a0.y, a1.x, a1.y};
}

__device__ __forceinline__ void stencil_pair(const float2* __restrict__ u, float2* __restrict__ y,
                                             const float* __restrict__ k2, const float2* __restrict__ cE,
                                             const float2* __restrict__ cW, const float2* __restrict__ cN,
                                             const float2* __restrict__ cS, const float2* __restrict__ dx,
                                             const float2* __restrict__ dy, int conj_diag, int nx, int ny,
                                             int64_t p) {
    ((float4*)y)[p >> 1] = stencil_pair_value(u, k2, cE, cW, cN, cS, dx, dy, conj_diag, nx, ny, p);
}

}  // namespace hz
