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

// The same operator for the two adjacent points (p, p + 1) = (gi, gi + 1) of one row, gi even,
// nx even, u / y 16-byte aligned: the centre, north and south pairs are 16-byte loads, the west
// and east neighbours 8-byte loads (zero outside the grid), the result one 16-byte store. Same
// term order as stencil_tile.
__device__ __forceinline__ void stencil_pair(const float2* __restrict__ u, float2* __restrict__ y,
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
    ((float4*)y)[q] = float4{a0.x, a0.y, a1.x, a1.y};
}

}  // namespace hz
