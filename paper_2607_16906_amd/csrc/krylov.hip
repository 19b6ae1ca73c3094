// Arnoldi and least-squares kernels of flexible GMRES (Algorithm 1, eq. (4), eq. (13)).
//
// Vectors are FP32 or FP64 complex; every inner product and norm accumulates in
// FP64, with deterministic two-stage reductions: each block writes one partial
// per quantity, and a separate pass sums the partials in a fixed order.
// Orthogonalisation is classical Gram-Schmidt with one reorthogonalisation
// (the same Hessenberg column as modified Gram-Schmidt in exact arithmetic):
//   pass 1: h1 = V^H w (and ||w||^2),  pass 2: w -= V h1, h2 = V^H w,
//   pass 3: w -= V h2 (and ||w||^2);   h = h1 + h2, h_{j+1,j} = ||w||.
// The Hessenberg least-squares problem is kept in FP64 with complex Givens
// rotations: for (a, b) = (h_jj, h_{j+1,j}), rho = sqrt(|a|^2 + |b|^2),
// c = |a| / rho, s = (a / |a|) conj(b) / rho (s = 1 when a = 0), and the pair
// (x, y) maps to (c x + s y, -conj(s) x + c y); the residual norm is |g_{j+1}|.
#include <algorithm>
#include <cmath>

#include "krylov.h"
#include "krylov_impl.h"
#include "problem.h"
#include "stencil_impl.h"

namespace hz {

Split krylov_split(int64_t n) {
    int64_t nblk = (n + KT - 1) / KT;
    if (nblk > 1024) nblk = 1024;
    if (nblk < 1) nblk = 1;
    int64_t per = (n + nblk - 1) / nblk;
    per = (per + KT - 1) / KT * KT;
    nblk = (n + per - 1) / per;
    if (nblk < 1) nblk = 1;
    return Split{(int)nblk, per};
}

template <typename C>
__global__ __launch_bounds__(KT) void k_norm_partials(const C* __restrict__ x, int64_t n, int64_t per,
                                                      double2* __restrict__ part, int ldp, int slot,
                                                      const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t p0 = blockIdx.x * per, p1 = min(n, p0 + per);
    norm_body(x, p0, p1, part + (int64_t)blockIdx.x * ldp + slot);
}

template <typename C>
__global__ __launch_bounds__(KT) void k_dots(const C* __restrict__ V, int64_t ldv, int nv,
                                             const C* __restrict__ w, int64_t n, int64_t per,
                                             double2* __restrict__ part, int ldp, int with_norm,
                                             const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t p0 = blockIdx.x * per, p1 = min(n, p0 + per);
    double2* mine = part + (int64_t)blockIdx.x * ldp;
    dots_body(V, ldv, nv, w, p0, p1, mine);
    if (with_norm) norm_body(w, p0, p1, mine + nv);
}

// w = A z evaluated pointwise over the block's index range (neighbours read through the cache,
// zero outside the grid; same term order as the tiled stencil), then the pass-1 sums of k_dots
// with the norm: part[b][i] = block sum of conj(V_i) w, part[b][nv] = ||w||^2.
// TWO (delayed reorthogonalisation): the sums are taken against both v~ = V_{nv-1} and w,
// part[b][i] = conj(V_i) v~, part[b][nv + i] = conj(V_i) w (i < nv), part[b][2 nv] = ||w||^2.
template <typename C, bool TWO>
__global__ __launch_bounds__(KT) void k_stencil_dots(const C* __restrict__ z, StencilCoef sc, int nx, int ny,
                                                     const C* __restrict__ V, int64_t ldv, int nv,
                                                     C* __restrict__ w, int64_t n, int64_t per,
                                                     double2* __restrict__ part, int ldp,
                                                     const int* __restrict__ skip, int pairs) {
    using T = decltype(C{}.x);
    if (skip && *skip) return;
    const C* __restrict__ cE = (const C*)sc.E;
    const C* __restrict__ cW = (const C*)sc.W;
    const C* __restrict__ cN = (const C*)sc.N;
    const C* __restrict__ cS = (const C*)sc.S;
    const C* __restrict__ dxv = (const C*)sc.dx;
    const C* __restrict__ dyv = (const C*)sc.dy;
    const T* __restrict__ k2 = (const T*)sc.k2;
    const int64_t p0 = blockIdx.x * per, p1 = min(n, p0 + per);
    if constexpr (std::is_same<C, float2>::value) {
        if (pairs) {   // two points per lane (nx even, aligned vectors, even block start)
            for (int64_t p = p0 + 2 * threadIdx.x; p < p1; p += 2 * KT)
                stencil_pair(z, w, k2, cE, cW, cN, cS, dxv, dyv, sc.conj_diag, nx, ny, p);
            __syncthreads();
            double2* mine = part + (int64_t)blockIdx.x * ldp;
            if constexpr (TWO) {
                dots2_body(V, ldv, nv, V + (int64_t)(nv - 1) * ldv, (const C*)w, p0, p1, mine, nv);
                norm_body((const C*)w, p0, p1, mine + 2 * nv);
            } else {
                dots_body(V, ldv, nv, (const C*)w, p0, p1, mine);
                norm_body((const C*)w, p0, p1, mine + nv);
            }
            return;
        }
    }
    const C zero{0, 0};
    for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
        const int gj = (int)(p / nx), gi = (int)(p - (int64_t)gj * nx);
        const C dxi = dxv[gi], dyj = dyv[gj];
        C d = C{k2[p] - dxi.x - dyj.x, -dxi.y - dyj.y};
        if (sc.conj_diag) d.y = -d.y;
        C acc = cmul(d, z[p]);
        acc = cadd(acc, cmul(cE[gi], gi + 1 < nx ? z[p + 1] : zero));
        acc = cadd(acc, cmul(cW[gi], gi > 0 ? z[p - 1] : zero));
        acc = cadd(acc, cmul(cN[gj], gj + 1 < ny ? z[p + nx] : zero));
        acc = cadd(acc, cmul(cS[gj], gj > 0 ? z[p - nx] : zero));
        w[p] = acc;
    }
    __syncthreads();   // the sweeps below may read points written by other threads of the block
    double2* mine = part + (int64_t)blockIdx.x * ldp;
    if constexpr (TWO) {
        dots2_body(V, ldv, nv, V + (int64_t)(nv - 1) * ldv, (const C*)w, p0, p1, mine, nv);
        norm_body((const C*)w, p0, p1, mine + 2 * nv);
        return;
    }
    dots_body(V, ldv, nv, (const C*)w, p0, p1, mine);
    norm_body((const C*)w, p0, p1, mine + nv);
}

constexpr int UPD_REG = 32;   // vectors held in registers by the single-pass first update
constexpr int UPD_SPLIT4 = 24; // up to this many vectors pass 2 splits them over 4 wavefronts

// w = A z and the pass-1 sums for FP32 vectors read as point pairs (even row length, 16-byte
// aligned vectors, even stride), with the basis split over the NW wavefronts of the block
// (wavefront q holds vectors [q G, q G + G), G = ceil(nv / NW) <= GMAX). Per tile of NW x 64 pairs
// wavefront q evaluates the operator on pairs [64 q, 64 q + 64) of the tile (same term order as the
// tiled stencil), stores them and puts them in LDS (double-buffered, one barrier per tile); then
// each wavefront accumulates conj(V_i) w over the whole tile for its own vectors, reduced within
// the wavefront. ||w||^2 is summed by the wavefront that evaluated each pair, then over the
// wavefronts in order. Writes the same partial layout as k_stencil_dots<float2, false>.
template <int GMAX, int NW>
__global__ __launch_bounds__(NW * 64) void k_stencil_dots_split(const float2* __restrict__ z, StencilCoef sc,
                                                                int nx, int ny, const float2* __restrict__ V,
                                                                int64_t ldv, int nv, float2* __restrict__ w,
                                                                int64_t n, int64_t per, double2* __restrict__ part,
                                                                int ldp, const int* __restrict__ skip) {
    const int skipped = skip ? *skip : 0;   // tested once the first tile's loads are in flight
    const int64_t p0 = blockIdx.x * per, p1 = min(n, p0 + per);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = threadIdx.x & 63;
    const int G = (nv + NW - 1) / NW;
    const int i0 = wv * G;
    const int cnt = max(0, min(G, nv - i0));
    __shared__ float4 shw[2][NW][64];
    __shared__ double red[NW];
    double ar[GMAX], ai[GMAX];
#pragma unroll
    for (int q = 0; q < GMAX; ++q) ar[q] = ai[q] = 0.0;
    double nacc = 0.0;
    const int64_t npair = (p1 - p0) >> 1;   // p0 and p1 are even on this path
    const int64_t q0 = p0 >> 1, hv = ldv >> 1;
    const float4* __restrict__ V4 = (const float4*)V;
    int buf = 0;
    for (int64_t k0 = 0; k0 < npair; k0 += NW * 64, buf ^= 1) {
        const int64_t k = k0 + wv * 64 + ln;
        float4 a{0.f, 0.f, 0.f, 0.f};
        if (k < npair)
            a = stencil_pair_value(z, (const float*)sc.k2, (const float2*)sc.E, (const float2*)sc.W,
                                   (const float2*)sc.N, (const float2*)sc.S, (const float2*)sc.dx,
                                   (const float2*)sc.dy, sc.conj_diag, nx, ny, p0 + 2 * k);
        asm volatile("" ::: "memory");
        if (k0 == 0 && skipped) return;   // uniform over the block; nothing written yet
        if (k < npair) {
            ((float4*)w)[q0 + k] = a;
            nacc += (double)a.x * a.x + (double)a.y * a.y + (double)a.z * a.z + (double)a.w * a.w;
        }
        shw[buf][wv][ln] = a;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NW; ++r) {
            const int64_t kr = k0 + r * 64 + ln;
            if (kr >= npair) break;
            const float4 wp = shw[buf][r][ln];
            float4 vr[GMAX];
#pragma unroll
            for (int q = 0; q < GMAX; ++q)
                if (q < cnt) vr[q] = V4[(int64_t)(i0 + q) * hv + q0 + kr];
#pragma unroll
            for (int q = 0; q < GMAX; ++q)
                if (q < cnt) {
                    const float4 v = vr[q];
                    ar[q] += (double)v.x * wp.x + (double)v.y * wp.y + (double)v.z * wp.z + (double)v.w * wp.w;
                    ai[q] += (double)v.x * wp.y - (double)v.y * wp.x + (double)v.z * wp.w - (double)v.w * wp.z;
                }
        }
    }
    double2* mine = part + (int64_t)blockIdx.x * ldp;
#pragma unroll
    for (int g0 = 0; g0 < GMAX; g0 += IC) {
        if (g0 >= cnt) break;
        double (&sr)[IC] = *reinterpret_cast<double (*)[IC]>(&ar[g0]);
        double (&si)[IC] = *reinterpret_cast<double (*)[IC]>(&ai[g0]);
        wave_store8(sr, si, mine + i0 + g0, cnt - g0);
    }
    nacc = wave_sum(nacc);
    if (ln == 0) red[wv] = nacc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int r = 0; r < NW; ++r) t += red[r];
        mine[nv] = double2{t, 0.0};
    }
}

// Pass 2 of the orthogonalisation for FP32 vectors read as point pairs (16-byte aligned, even
// stride), with V read once for any nv <= NW GMAX: the vectors are split over the NW wavefronts of
// the block (wavefront q holds vectors [q G, q G + G), G = ceil(nv / NW), in registers). Per tile of
// 64 pairs each wavefront forms its part of V h; the NW parts and w meet in LDS (double-buffered,
// one barrier per tile); every wavefront forms the same w' = w - (sum of the parts in wavefront
// order), wavefront 0 stores it, and each wavefront accumulates conj(V_i) w' for its own vectors,
// reduced within the wavefront. Writes the same partial layout as k_update<float2, 1>.
template <int GMAX, int NW>
__global__ __launch_bounds__(NW * 64) void k_upd1_split(const float2* __restrict__ V, int64_t ldv, int nv,
                                                   const double2* __restrict__ h, float2* __restrict__ w,
                                                   int64_t n, int64_t per, double2* __restrict__ part, int ldp,
                                                   const int* __restrict__ skip) {
    const int skipped = skip ? *skip : 0;   // tested once the first tile's loads are in flight
    const int64_t p0 = blockIdx.x * per, p1 = min(n, p0 + per);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = threadIdx.x & 63;
    const int G = (nv + NW - 1) / NW;
    const int i0 = wv * G;
    const int cnt = max(0, min(G, nv - i0));
    __shared__ double4 sh[2][NW][64];
    __shared__ float4 shw[2][64];
    double ar[GMAX], ai[GMAX];
#pragma unroll
    for (int q = 0; q < GMAX; ++q) ar[q] = ai[q] = 0.0;
    const int64_t len = p1 - p0;
    // pairs, the last one a single point when len is odd (an odd-length vector in a basis of even
    // stride; the solver's bases have stride n, and an odd n takes k_update instead)
    const int64_t nunit = (len + 1) >> 1;
    int buf = 0;
    for (int64_t k0 = 0; k0 < nunit; k0 += 64, buf ^= 1) {
        const int64_t k = k0 + ln;
        const bool valid = k < nunit;
        const bool half = 2 * k + 1 == len;
        const int64_t p = p0 + 2 * k;
        float4 vr[GMAX];
#pragma unroll
        for (int q = 0; q < GMAX; ++q) {
            vr[q] = float4{0.f, 0.f, 0.f, 0.f};
            if (q < cnt && valid) {
                const float2* src = V + (int64_t)(i0 + q) * ldv + p;
                if (half) {
                    const float2 t = src[0];
                    vr[q] = float4{t.x, t.y, 0.f, 0.f};
                } else {
                    vr[q] = *(const float4*)src;
                }
            }
        }
        if (wv == 0) {
            float4 a{0.f, 0.f, 0.f, 0.f};
            if (valid) {
                if (half) {
                    const float2 t = w[p];
                    a = float4{t.x, t.y, 0.f, 0.f};
                } else {
                    a = *(const float4*)(w + p);
                }
            }
            shw[buf][ln] = a;
        }
        double sx = 0.0, sy = 0.0, tx = 0.0, ty = 0.0;
#pragma unroll
        for (int q = 0; q < GMAX; ++q)
            if (q < cnt) {
                const float4 v = vr[q];
                const double2 hi = h[i0 + q];   // wavefront-uniform: scalar loads
                sx += (double)v.x * hi.x - (double)v.y * hi.y;
                sy += (double)v.x * hi.y + (double)v.y * hi.x;
                tx += (double)v.z * hi.x - (double)v.w * hi.y;
                ty += (double)v.z * hi.y + (double)v.w * hi.x;
            }
        sh[buf][wv][ln] = double4{sx, sy, tx, ty};
        if (k0 == 0 && skipped) return;   // uniform over the block; nothing written yet
        __syncthreads();
        const float4 a = shw[buf][ln];
        double ax = a.x, ay = a.y, bx = a.z, by = a.w;
#pragma unroll
        for (int r = 0; r < NW; ++r) {
            const double4 s = sh[buf][r][ln];
            ax -= s.x;
            ay -= s.y;
            bx -= s.z;
            by -= s.w;
        }
        const float4 wp{(float)ax, (float)ay, half ? 0.f : (float)bx, half ? 0.f : (float)by};
        if (wv == 0 && valid) {
            if (half)
                w[p] = float2{wp.x, wp.y};
            else
                *(float4*)(w + p) = wp;
        }
#pragma unroll
        for (int q = 0; q < GMAX; ++q)
            if (q < cnt) {
                const float4 v = vr[q];
                ar[q] += (double)v.x * wp.x + (double)v.y * wp.y + (double)v.z * wp.z + (double)v.w * wp.w;
                ai[q] += (double)v.x * wp.y - (double)v.y * wp.x + (double)v.z * wp.w - (double)v.w * wp.z;
            }
    }
    double2* mine = part + (int64_t)blockIdx.x * ldp + i0;
#pragma unroll
    for (int g0 = 0; g0 < GMAX; g0 += IC) {
        if (g0 >= cnt) break;
        double (&sr)[IC] = *reinterpret_cast<double (*)[IC]>(&ar[g0]);
        double (&si)[IC] = *reinterpret_cast<double (*)[IC]>(&ai[g0]);
        wave_store8(sr, si, mine + g0, cnt - g0);
    }
}

template <typename C, int MODE>
__global__ __launch_bounds__(KT) void k_update(const C* __restrict__ V, int64_t ldv, int nv,
                                               const double2* __restrict__ h, C* __restrict__ w, int64_t n,
                                               int64_t per, double2* __restrict__ part, int ldp,
                                               const int* __restrict__ skip) {
    const int64_t p0 = blockIdx.x * per, p1 = min(n, p0 + per);
    {
        // the step-skip flag's load overlaps that of the block's first point of w (which
        // brings its line into the cache for the loops below); nothing is written before the test
        const int skipped = skip ? *skip : 0;
        const int64_t pf = min(p0 + (int64_t)threadIdx.x, n - 1);
        const C warm = w[pf];
        asm volatile("" ::"v"(warm.x));
        if (skipped) return;
    }
    if (MODE == 1 && nv <= UPD_REG) {
        // single pass: the vectors read for the update of a point stay in registers for the sums
        // conj(V_i) w of the second Gram-Schmidt pass (V is read once)
        double ar[UPD_REG], ai[UPD_REG];
#pragma unroll
        for (int i = 0; i < UPD_REG; ++i) ar[i] = ai[i] = 0.0;
        for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
            C vr[UPD_REG];
#pragma unroll
            for (int i = 0; i < UPD_REG; ++i)
                if (i < nv) vr[i] = V[(int64_t)i * ldv + p];
            const C w0 = w[p];
            double ax = w0.x, ay = w0.y;
#pragma unroll
            for (int i = 0; i < UPD_REG; ++i)
                if (i < nv) {
                    const double2 hi = h[i];
                    ax -= (double)vr[i].x * hi.x - (double)vr[i].y * hi.y;
                    ay -= (double)vr[i].x * hi.y + (double)vr[i].y * hi.x;
                }
            const C wp = from_d2<C>(double2{ax, ay});
            w[p] = wp;
#pragma unroll
            for (int i = 0; i < UPD_REG; ++i)
                if (i < nv) {
                    ar[i] += (double)vr[i].x * wp.x + (double)vr[i].y * wp.y;
                    ai[i] += (double)vr[i].x * wp.y - (double)vr[i].y * wp.x;
                }
        }
        // each wavefront reduces its lanes group by group, the 4 wavefront totals meet in LDS
        double2* mine = part + (int64_t)blockIdx.x * ldp;
        __shared__ double red[KT / 64][2 * UPD_REG];
        const int wv = threadIdx.x >> 6;
#pragma unroll
        for (int i0 = 0; i0 < UPD_REG; i0 += IC) {
            if (i0 >= nv) break;
            double (&sr)[IC] = *reinterpret_cast<double (*)[IC]>(&ar[i0]);
            double (&si)[IC] = *reinterpret_cast<double (*)[IC]>(&ai[i0]);
            int idx;
            const double v = wave_reduce8(sr, si, &idx);
            if ((threadIdx.x & 3) == 0) red[wv][2 * i0 + idx] = v;
        }
        __syncthreads();
        if (threadIdx.x < 2 * nv) {
            double t = 0;
#pragma unroll
            for (int k = 0; k < KT / 64; ++k) t += red[k][threadIdx.x];
            ((double*)mine)[threadIdx.x] = t;
        }
        return;
    }
    update_body(V, ldv, nv, h, w, p0, p1);
    __syncthreads();   // the sweeps below may read points written by other threads of the block
    double2* mine = part + (int64_t)blockIdx.x * ldp;
    if (MODE == 1) dots_body(V, ldv, nv, w, p0, p1, mine);
    if (MODE == 2) norm_body(w, p0, p1, mine);
}

// one block per output value
__global__ __launch_bounds__(KT) void k_finalize(const double2* __restrict__ part, int nblk, int ldp,
                                                 double2* __restrict__ out, const int* __restrict__ skip) {
    const int skipped = skip ? *skip : 0;   // its load overlaps those of the partials
    const double2 v = block_sum_slot(part, nblk, ldp, blockIdx.x);
    if (threadIdx.x == 0 && !skipped) out[blockIdx.x] = v;
}


// ||b|| from the partials in slot 0; resets the counters.

__global__ void k_init_state(SolveState* st, const double2* part, int nblk, int ldp, double tol, int m,
                             int hist_cap) {
    init_state_body(st, part, nblk, ldp, tol, m, hist_cap);
}


__global__ void k_cycle_start(SolveState* st, const double* __restrict__ rpart, int nparts, double2* g, int m) {
    cycle_start_body(st, rpart, nparts, g, m);
}

template <typename C>
__global__ __launch_bounds__(KT) void k_cast_scale(const double2* __restrict__ r, C* __restrict__ v, int64_t n,
                                                   const SolveState* __restrict__ st) {
    if (st->stop) return;
    const double s = st->inv_beta;
    for (int64_t p = (int64_t)blockIdx.x * KT + threadIdx.x; p < n; p += (int64_t)gridDim.x * KT) {
        const double2 a = r[p];
        v[p] = from_d2<C>(double2{a.x * s, a.y * s});
    }
}

template <typename C>
__global__ __launch_bounds__(KT) void k_scale(C* __restrict__ v, int64_t n, const double* __restrict__ inv,
                                              const int* __restrict__ skip) {
    if (skip && *skip) return;
    const double s = *inv;
    for (int64_t p = (int64_t)blockIdx.x * KT + threadIdx.x; p < n; p += (int64_t)gridDim.x * KT) {
        const C a = v[p];
        v[p] = from_d2<C>(double2{a.x * s, a.y * s});
    }
}


__global__ void k_arnoldi_finish(SolveState* st, double2* R, double* cs, double2* sn, double2* g,
                                 const double2* h1, const double2* h2, const double2* part, int nblk, int ldp,
                                 int j, double* hist) {
    arnoldi_finish_body(st, R, cs, sn, g, h1, h2, part, nblk, ldp, j, hist);
}


__global__ void k_backsolve(SolveState* st, const double2* R, const double2* g, double2* y) {
    backsolve_body(st, R, g, y);
}

template <typename C>
__global__ __launch_bounds__(KT) void k_xupdate(const C* __restrict__ Z, int64_t ldz, double2* __restrict__ x,
                                                int64_t n, const double2* __restrict__ y,
                                                const SolveState* __restrict__ st) {
    const int k = st->k;
    if (k == 0) return;
    for (int64_t p = (int64_t)blockIdx.x * KT + threadIdx.x; p < n; p += (int64_t)gridDim.x * KT) {
        double2 a = x[p];
        for (int i = 0; i < k; ++i) {
            const C z = Z[(int64_t)i * ldz + p];
            const double2 yi = y[i];
            a.x += (double)z.x * yi.x - (double)z.y * yi.y;
            a.y += (double)z.x * yi.y + (double)z.y * yi.x;
        }
        x[p] = a;
    }
}

// ------------------------------------------------------------------ launchers

static unsigned grid_for(int64_t n) {
    int64_t g = (n + KT - 1) / KT;
    if (g > 2048) g = 2048;
    return (unsigned)(g < 1 ? 1 : g);
}

int launch_norm_partials(bool c128, const void* x, int64_t n, Split sp, double2* part, int ldp, int slot,
                         const int* skip, hipStream_t s) {
    if (c128)
        hipLaunchKernelGGL(k_norm_partials<double2>, dim3(sp.nblk), dim3(KT), 0, s, (const double2*)x, n,
                           sp.per_block, part, ldp, slot, skip);
    else
        hipLaunchKernelGGL(k_norm_partials<float2>, dim3(sp.nblk), dim3(KT), 0, s, (const float2*)x, n,
                           sp.per_block, part, ldp, slot, skip);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_finalize(const double2* part, int nblk, int ldp, int cnt, double2* out, const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(cnt), dim3(KT), 0, s, part, nblk, ldp, out, skip);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_dots(bool c128, const void* V, int64_t ldv, int nv, const void* w, int64_t n, Split sp,
                double2* part, int ldp, bool with_norm, const int* skip, hipStream_t s) {
    if (c128)
        hipLaunchKernelGGL(k_dots<double2>, dim3(sp.nblk), dim3(KT), 0, s, (const double2*)V, ldv, nv,
                           (const double2*)w, n, sp.per_block, part, ldp, with_norm ? 1 : 0, skip);
    else
        hipLaunchKernelGGL(k_dots<float2>, dim3(sp.nblk), dim3(KT), 0, s, (const float2*)V, ldv, nv,
                           (const float2*)w, n, sp.per_block, part, ldp, with_norm ? 1 : 0, skip);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_stencil_dots(const hz_problem* p, bool c128, const void* z, const void* V, int64_t ldv, int nv,
                        void* w, Split sp, double2* part, int ldp, const int* skip, hipStream_t s, bool two) {
    if (is_spectral(p)) {
        // the Fourier-differentiation operator, then the Gram-Schmidt sums as a separate pass
        if (two) {
            set_error("fgmres: the spectral operator runs with ortho = 0");
            return HZ_ERR_ARG;
        }
        HZ_TRY(launch_spectral(p, c128, false, z, w, s, skip));
        return launch_dots(c128, V, ldv, nv, w, p->n, sp, part, ldp, true, skip, s);
    }
    const StencilCoef sc = stencil_coef(p, c128, false);
    // the pair form needs even block starts (per_block is a multiple of the block size) and an
    // even row length
    const int pairs = !c128 && stencil_pairs_ok(p, z, w) && (sp.per_block & 1) == 0 ? 1 : 0;
#define HZ_SD(C, TW, PR)                                                                                       \
    hipLaunchKernelGGL((k_stencil_dots<C, TW>), dim3(sp.nblk), dim3(KT), 0, s, (const C*)z, sc, p->nxt, p->nyt, \
                       (const C*)V, ldv, nv, (C*)w, p->n, sp.per_block, part, ldp, skip, PR)
    const bool vpairs = (ldv & 1) == 0 && (((uintptr_t)V) & 15) == 0;
    if (c128) {
        if (two) HZ_SD(double2, true, 0);
        else HZ_SD(double2, false, 0);
    } else if (!two && pairs && vpairs && nv <= 32) {
        hipLaunchKernelGGL((k_stencil_dots_split<8, 4>), dim3(sp.nblk), dim3(256), 0, s, (const float2*)z, sc,
                           p->nxt, p->nyt, (const float2*)V, ldv, nv, (float2*)w, p->n, sp.per_block, part, ldp,
                           skip);
    } else if (!two && pairs && vpairs && nv <= 64) {
        hipLaunchKernelGGL((k_stencil_dots_split<8, 8>), dim3(sp.nblk), dim3(512), 0, s, (const float2*)z, sc,
                           p->nxt, p->nyt, (const float2*)V, ldv, nv, (float2*)w, p->n, sp.per_block, part, ldp,
                           skip);
    } else {
        if (two) HZ_SD(float2, true, pairs);
        else HZ_SD(float2, false, pairs);
    }
#undef HZ_SD
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

// Delayed-reorthogonalisation update of step j (one pass over q_0 .. q_{j-1}): slot j (v~)
// becomes q_j = (v~ - sum_i a_i q_i) / nu and slot j + 1 (w) becomes w - sum_i b_i q_i - h_jj q_j,
// with q_j as stored; coef = [a_0 .. a_{j-1}, b_0 .. b_{j-1}, h_jj, (1 / nu, 0)]. Each block writes
// the squared norm of its part of the new slot j + 1 (as stored) to part[b * ldp].x: the next
// network input's scale.
template <typename C>
__global__ __launch_bounds__(KT) void k_update_lag(C* __restrict__ V, int64_t ldv, int j,
                                                   const double2* __restrict__ coef, int64_t n, int64_t per,
                                                   double2* __restrict__ part, int ldp,
                                                   const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t p0 = blockIdx.x * per, p1 = min(n, p0 + per);
    C* __restrict__ vt = V + (int64_t)j * ldv;
    C* __restrict__ w = V + (int64_t)(j + 1) * ldv;
    const double inv_nu = coef[2 * j + 1].x;
    const double2 h = coef[2 * j];
    double nw[1] = {0.0}, zz[1] = {0.0};
    bool done = false;
    if constexpr (std::is_same<C, float2>::value) {
        if (pair_ok<C>(V, V, ldv, p0)) {
            float4* __restrict__ v4 = (float4*)(vt + p0);
            float4* __restrict__ w4 = (float4*)(w + p0);
            const int64_t npair = (p1 - p0) >> 1;
            for (int64_t k = threadIdx.x; k < npair; k += KT) {
                const float4 a0 = v4[k], b0 = w4[k];
                double vx = a0.x, vy = a0.y, vz = a0.z, vw = a0.w;
                double wx = b0.x, wy = b0.y, wz = b0.z, ww = b0.w;
                for (int i = 0; i < j; ++i) {
                    const float4 q = ((const float4*)(V + (int64_t)i * ldv + p0))[k];
                    const double2 a = coef[i], b = coef[j + i];
                    vx -= (double)q.x * a.x - (double)q.y * a.y;
                    vy -= (double)q.x * a.y + (double)q.y * a.x;
                    vz -= (double)q.z * a.x - (double)q.w * a.y;
                    vw -= (double)q.z * a.y + (double)q.w * a.x;
                    wx -= (double)q.x * b.x - (double)q.y * b.y;
                    wy -= (double)q.x * b.y + (double)q.y * b.x;
                    wz -= (double)q.z * b.x - (double)q.w * b.y;
                    ww -= (double)q.z * b.y + (double)q.w * b.x;
                }
                const float4 qj{(float)(vx * inv_nu), (float)(vy * inv_nu), (float)(vz * inv_nu), (float)(vw * inv_nu)};
                wx -= (double)qj.x * h.x - (double)qj.y * h.y;
                wy -= (double)qj.x * h.y + (double)qj.y * h.x;
                wz -= (double)qj.z * h.x - (double)qj.w * h.y;
                ww -= (double)qj.z * h.y + (double)qj.w * h.x;
                const float4 wn{(float)wx, (float)wy, (float)wz, (float)ww};
                v4[k] = qj;
                w4[k] = wn;
                nw[0] += (double)wn.x * wn.x + (double)wn.y * wn.y + (double)wn.z * wn.z + (double)wn.w * wn.w;
            }
            done = ((p1 - p0) & 1) == 0;
            if (!done) {
                // the odd last point of the range, by one thread
                if (threadIdx.x == KT - 1) {
                    const int64_t p = p1 - 1;
                    const C a0 = vt[p], b0 = w[p];
                    double vx = a0.x, vy = a0.y, wx = b0.x, wy = b0.y;
                    for (int i = 0; i < j; ++i) {
                        const C q = V[(int64_t)i * ldv + p];
                        const double2 a = coef[i], b = coef[j + i];
                        vx -= (double)q.x * a.x - (double)q.y * a.y;
                        vy -= (double)q.x * a.y + (double)q.y * a.x;
                        wx -= (double)q.x * b.x - (double)q.y * b.y;
                        wy -= (double)q.x * b.y + (double)q.y * b.x;
                    }
                    const C qj = from_d2<C>(double2{vx * inv_nu, vy * inv_nu});
                    wx -= (double)qj.x * h.x - (double)qj.y * h.y;
                    wy -= (double)qj.x * h.y + (double)qj.y * h.x;
                    const C wn = from_d2<C>(double2{wx, wy});
                    vt[p] = qj;
                    w[p] = wn;
                    nw[0] += (double)wn.x * wn.x + (double)wn.y * wn.y;
                }
                done = true;
            }
        }
    }
    if (!done) {
        for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
            const C a0 = vt[p], b0 = w[p];
            double vx = a0.x, vy = a0.y, wx = b0.x, wy = b0.y;
            for (int i = 0; i < j; ++i) {
                const C q = V[(int64_t)i * ldv + p];
                const double2 a = coef[i], b = coef[j + i];
                vx -= (double)q.x * a.x - (double)q.y * a.y;
                vy -= (double)q.x * a.y + (double)q.y * a.x;
                wx -= (double)q.x * b.x - (double)q.y * b.y;
                wy -= (double)q.x * b.y + (double)q.y * b.x;
            }
            const C qj = from_d2<C>(double2{vx * inv_nu, vy * inv_nu});
            wx -= (double)qj.x * h.x - (double)qj.y * h.y;
            wy -= (double)qj.x * h.y + (double)qj.y * h.x;
            const C wn = from_d2<C>(double2{wx, wy});
            vt[p] = qj;
            w[p] = wn;
            nw[0] += (double)wn.x * wn.x + (double)wn.y * wn.y;
        }
    }
    block_store<1>(nw, zz, part + (int64_t)blockIdx.x * ldp, 1);
}

__global__ void k_arnoldi_lag(SolveState* st, double2* R, double* cs, double2* sn, double2* g, double2* pend,
                              double2* colb, double2* coef, double* sc, const double2* red, int j, int tail,
                              double* hist) {
    arnoldi_lag_body(st, R, cs, sn, g, pend, colb, coef, sc, red, j, tail, hist);
}

int launch_update_lag(bool c128, void* V, int64_t ldv, int j, const double2* coef, int64_t n, Split sp,
                      double2* part, int ldp, const int* skip, hipStream_t s) {
    if (c128)
        hipLaunchKernelGGL(k_update_lag<double2>, dim3(sp.nblk), dim3(KT), 0, s, (double2*)V, ldv, j, coef, n,
                           sp.per_block, part, ldp, skip);
    else
        hipLaunchKernelGGL(k_update_lag<float2>, dim3(sp.nblk), dim3(KT), 0, s, (float2*)V, ldv, j, coef, n,
                           sp.per_block, part, ldp, skip);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_arnoldi_lag(KrylovBufs& kb, int j, bool tail, hipStream_t s) {
    hipLaunchKernelGGL(k_arnoldi_lag, dim3(1), dim3(64), 0, s, kb.st, kb.R, kb.cs, kb.sn, kb.g, kb.pend, kb.colb,
                       kb.coef, kb.lag_sc, kb.h1, j, tail ? 1 : 0, kb.hist);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_update(bool c128, const void* V, int64_t ldv, int nv, const double2* h, void* w, int64_t n,
                  Split sp, double2* part, int ldp, int mode, const int* skip, hipStream_t s) {
#define HZ_UPD(C, M)                                                                                   \
    hipLaunchKernelGGL((k_update<C, M>), dim3(sp.nblk), dim3(KT), 0, s, (const C*)V, ldv, nv, h, (C*)w, n, \
                       sp.per_block, part, ldp, skip)
    if (c128) {
        if (mode == 0) HZ_UPD(double2, 0);
        else if (mode == 1) HZ_UPD(double2, 1);
        else HZ_UPD(double2, 2);
    } else {
        // pass 2 with the vectors split over the wavefronts where that measured faster (short
        // bases, and bases too long for k_update's single-pass register form)
        const bool pairs = (ldv & 1) == 0 && ((((uintptr_t)V) | ((uintptr_t)w)) & 15) == 0;
        if (mode == 1 && pairs && nv <= UPD_SPLIT4)
            hipLaunchKernelGGL((k_upd1_split<8, 4>), dim3(sp.nblk), dim3(256), 0, s, (const float2*)V, ldv, nv, h,
                               (float2*)w, n, sp.per_block, part, ldp, skip);
        else if (mode == 1 && pairs && nv > UPD_REG && nv <= 64)
            hipLaunchKernelGGL((k_upd1_split<8, 8>), dim3(sp.nblk), dim3(512), 0, s, (const float2*)V, ldv, nv, h,
                               (float2*)w, n, sp.per_block, part, ldp, skip);
        else if (mode == 0) HZ_UPD(float2, 0);
        else if (mode == 1) HZ_UPD(float2, 1);
        else HZ_UPD(float2, 2);
    }
#undef HZ_UPD
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_init_state(KrylovBufs& kb, int nblk, double tol, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, kb.st, kb.part, nblk, kb.ldp, tol, m,
                       kb.hist_cap);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_arnoldi_finish(KrylovBufs& kb, int j, int nblk, bool reorth, hipStream_t s) {
    hipLaunchKernelGGL(k_arnoldi_finish, dim3(1), dim3(64), 0, s, kb.st, kb.R, kb.cs, kb.sn, kb.g, kb.h1,
                       reorth ? kb.h2 : nullptr, kb.part, nblk, kb.ldp, j, kb.hist);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_scale(bool c128, void* v, int64_t n, const double* inv, const int* skip, hipStream_t s) {
    if (c128)
        hipLaunchKernelGGL(k_scale<double2>, dim3(grid_for(n)), dim3(KT), 0, s, (double2*)v, n, inv, skip);
    else
        hipLaunchKernelGGL(k_scale<float2>, dim3(grid_for(n)), dim3(KT), 0, s, (float2*)v, n, inv, skip);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_cycle_start(KrylovBufs& kb, const double* resid_part, int nparts, hipStream_t s) {
    // m is read on the device from the state; pass the bound of g explicitly
    hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(64), 0, s, kb.st, resid_part, nparts, kb.g, kb.ldp - 2);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_cast_scale(bool c128, const double2* r, void* v, int64_t n, const SolveState* st, hipStream_t s) {
    if (c128)
        hipLaunchKernelGGL(k_cast_scale<double2>, dim3(grid_for(n)), dim3(KT), 0, s, r, (double2*)v, n, st);
    else
        hipLaunchKernelGGL(k_cast_scale<float2>, dim3(grid_for(n)), dim3(KT), 0, s, r, (float2*)v, n, st);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_backsolve(KrylovBufs& kb, hipStream_t s) {
    hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, s, kb.st, kb.R, kb.g, kb.y);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_xupdate(bool c128, const void* Z, int64_t ldz, double2* x, int64_t n, const KrylovBufs& kb,
                   hipStream_t s) {
    if (c128)
        hipLaunchKernelGGL(k_xupdate<double2>, dim3(grid_for(n)), dim3(KT), 0, s, (const double2*)Z, ldz, x, n,
                           kb.y, kb.st);
    else
        hipLaunchKernelGGL(k_xupdate<float2>, dim3(grid_for(n)), dim3(KT), 0, s, (const float2*)Z, ldz, x, n,
                           kb.y, kb.st);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

}  // namespace hz
