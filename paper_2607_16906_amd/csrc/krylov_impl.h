// Device bodies of the FP64-accumulating block reductions used by the Arnoldi kernels
// (shared by the single-system and the ragged-batch kernels).
#pragma once

#include <type_traits>

#include "common.h"
#include "krylov.h"

namespace hz {

constexpr int KT = 256;   // threads per block of the vector kernels
constexpr int IC = 8;     // inner products accumulated per sweep

// Sum NV pairs over the block and store the first cnt of them as out[q]. For NV >= 2 the
// 2 NV values are transposed through LDS: 256 / (2 NV) consecutive lanes own one value, each
// sums a strided slice of the 256 thread contributions, and the lanes combine with
// in-wavefront shuffles (fixed order, so the result is deterministic).
template <int NV>
__device__ __forceinline__ void block_store(double (&ar)[NV], double (&ai)[NV], double2* out, int cnt) {
    if constexpr (NV >= 2) {
        constexpr int NVAL = 2 * NV;
        constexpr int PER = KT / NVAL;          // lanes per value (<= 64)
        __shared__ double red[NVAL][KT];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            red[2 * q][threadIdx.x] = ar[q];
            red[2 * q + 1][threadIdx.x] = ai[q];
        }
        __syncthreads();
        const int v = threadIdx.x / PER, g = threadIdx.x % PER;
        double s = 0;
#pragma unroll
        for (int k = 0; k < KT / PER; ++k) s += red[v][g + PER * k];
#pragma unroll
        for (int o = PER / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (g == 0 && (v >> 1) < cnt) ((double*)out)[v] = s;
        __syncthreads();
    } else {
        __shared__ double red[KT / 64][2 * NV];
        const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double a = wave_sum(ar[q]), b = wave_sum(ai[q]);
            if (ln == 0) {
                red[wv][2 * q] = a;
                red[wv][2 * q + 1] = b;
            }
        }
        __syncthreads();
        if (threadIdx.x < cnt && threadIdx.x < NV) {
            double a = 0, b = 0;
#pragma unroll
            for (int w = 0; w < KT / 64; ++w) {
                a += red[w][2 * threadIdx.x];
                b += red[w][2 * threadIdx.x + 1];
            }
            out[threadIdx.x] = double2{a, b};
        }
        __syncthreads();
    }
}

// Sum IC = 8 complex values (16 doubles) over the 64 lanes of a wavefront with a transposing
// butterfly (each exchange halves what a lane carries: 8 + 4 + 2 + 1 + 1 + 1 shuffles instead of
// 16 x 6), fixed order. Afterwards lane l holds double number 8 b5 + 4 b4 + 2 b3 + b2 (bits of l)
// of the 16 (re, im, re, im, ...); returns it and its index.
__device__ __forceinline__ double wave_reduce8(const double (&ar)[IC], const double (&ai)[IC], int* idx) {
    static_assert(IC == 8, "wave_reduce8 reduces 8 complex values");
    const int ln = threadIdx.x & 63;
    const int b5 = (ln >> 5) & 1, b4 = (ln >> 4) & 1, b3 = (ln >> 3) & 1, b2 = (ln >> 2) & 1;
    double x[16];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        x[2 * q] = ar[q];
        x[2 * q + 1] = ai[q];
    }
    double y[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) y[k] = (b5 ? x[k + 8] : x[k]) + __shfl_xor(b5 ? x[k] : x[k + 8], 32, 64);
    double z[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) z[k] = (b4 ? y[k + 4] : y[k]) + __shfl_xor(b4 ? y[k] : y[k + 4], 16, 64);
    double u[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) u[k] = (b3 ? z[k + 2] : z[k]) + __shfl_xor(b3 ? z[k] : z[k + 2], 8, 64);
    double v = (b2 ? u[1] : u[0]) + __shfl_xor(b2 ? u[0] : u[1], 4, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 1, 64);
    *idx = 8 * b5 + 4 * b4 + 2 * b3 + b2;
    return v;
}

// part[q] = wavefront sum of (ar[q], ai[q]) for q < cnt (no LDS, no barrier)
__device__ __forceinline__ void wave_store8(const double (&ar)[IC], const double (&ai)[IC], double2* out, int cnt) {
    int idx;
    const double v = wave_reduce8(ar, ai, &idx);
    if ((threadIdx.x & 3) == 0 && (idx >> 1) < cnt) ((double*)out)[idx] = v;
}

// FP32 complex vectors with an even stride and 16-byte aligned bases are read two points per
// lane (one 16-byte load per vector): the pair path of the sweeps below.
template <typename C>
__device__ __forceinline__ bool pair_ok(const void* a, const void* b, int64_t ldv, int64_t p0) {
    if constexpr (std::is_same<C, float2>::value)
        return ((ldv | p0) & 1) == 0 && ((((uintptr_t)a) | ((uintptr_t)b)) & 15) == 0;
    return false;
}

// part[i] = sum over [p0, p1) of conj(V_i) w, i < nv, two points per lane
__device__ __forceinline__ void dots_body_pairs(const float2* __restrict__ V, int64_t ldv, int nv,
                                                const float2* __restrict__ w, int64_t p0, int64_t p1,
                                                double2* __restrict__ part) {
    const int64_t npair = (p1 - p0) >> 1;
    const float4* __restrict__ w4 = (const float4*)(w + p0);
    for (int i0 = 0; i0 < nv; i0 += IC) {
        double ar[IC], ai[IC];
#pragma unroll
        for (int q = 0; q < IC; ++q) ar[q] = ai[q] = 0.0;
        for (int64_t k = threadIdx.x; k < npair; k += KT) {
            const float4 a = w4[k];
#pragma unroll
            for (int q = 0; q < IC; ++q) {
                if (i0 + q < nv) {
                    const float4 v = ((const float4*)(V + (int64_t)(i0 + q) * ldv + p0))[k];
                    ar[q] += (double)v.x * a.x + (double)v.y * a.y + (double)v.z * a.z + (double)v.w * a.w;
                    ai[q] += (double)v.x * a.y - (double)v.y * a.x + (double)v.z * a.w - (double)v.w * a.z;
                }
            }
        }
        if (((p1 - p0) & 1) && threadIdx.x == KT - 1) {   // odd tail point
            const float2 a = w[p1 - 1];
#pragma unroll
            for (int q = 0; q < IC; ++q)
                if (i0 + q < nv) {
                    const float2 v = V[(int64_t)(i0 + q) * ldv + p1 - 1];
                    ar[q] += (double)v.x * a.x + (double)v.y * a.y;
                    ai[q] += (double)v.x * a.y - (double)v.y * a.x;
                }
        }
        block_store<IC>(ar, ai, part + i0, nv - i0);
    }
}

// Long bases (more than 2 IC vectors): wavefront wv takes the groups of IC vectors i0 = IC wv,
// IC (wv + 4), ... over all of the block's points and reduces each group within the wavefront,
// so the groups' loads and reductions overlap across the 4 wavefronts (no block barrier).
template <typename C>
__device__ __forceinline__ void dots_body_waves(const C* __restrict__ V, int64_t ldv, int nv,
                                                const C* __restrict__ w, int64_t p0, int64_t p1,
                                                double2* __restrict__ part) {
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const bool pairs = pair_ok<C>(V, w, ldv, p0);
    for (int i0 = wv * IC; i0 < nv; i0 += (KT / 64) * IC) {
        double ar[IC], ai[IC];
#pragma unroll
        for (int q = 0; q < IC; ++q) ar[q] = ai[q] = 0.0;
        if constexpr (std::is_same<C, float2>::value) {
            if (pairs) {
                const int64_t npair = (p1 - p0) >> 1;
                const float4* __restrict__ w4 = (const float4*)(w + p0);
                for (int64_t k = ln; k < npair; k += 64) {
                    const float4 a = w4[k];
#pragma unroll
                    for (int q = 0; q < IC; ++q) {
                        if (i0 + q < nv) {
                            const float4 v = ((const float4*)(V + (int64_t)(i0 + q) * ldv + p0))[k];
                            ar[q] += (double)v.x * a.x + (double)v.y * a.y + (double)v.z * a.z + (double)v.w * a.w;
                            ai[q] += (double)v.x * a.y - (double)v.y * a.x + (double)v.z * a.w - (double)v.w * a.z;
                        }
                    }
                }
                if (((p1 - p0) & 1) && ln == 63) {   // odd tail point
                    const float2 a = w[p1 - 1];
#pragma unroll
                    for (int q = 0; q < IC; ++q)
                        if (i0 + q < nv) {
                            const float2 v = V[(int64_t)(i0 + q) * ldv + p1 - 1];
                            ar[q] += (double)v.x * a.x + (double)v.y * a.y;
                            ai[q] += (double)v.x * a.y - (double)v.y * a.x;
                        }
                }
                wave_store8(ar, ai, part + i0, nv - i0);
                continue;
            }
        }
        for (int64_t p = p0 + ln; p < p1; p += 64) {
            const C wp = w[p];
#pragma unroll
            for (int q = 0; q < IC; ++q) {
                if (i0 + q < nv) {
                    const C v = V[(int64_t)(i0 + q) * ldv + p];
                    ar[q] += (double)v.x * wp.x + (double)v.y * wp.y;
                    ai[q] += (double)v.x * wp.y - (double)v.y * wp.x;
                }
            }
        }
        wave_store8(ar, ai, part + i0, nv - i0);
    }
}

// w -= sum_i V_i h_i (i in order) over points [p0, p1) of one KT-thread block: two points per lane
// with 16-byte loads and stores where the vectors allow it (pair_ok), else one; the basis loads of
// several i are in flight together.
template <typename C>
__device__ __forceinline__ void update_body(const C* __restrict__ V, int64_t ldv, int nv, const double2* __restrict__ h,
                                            C* __restrict__ w, int64_t p0, int64_t p1) {
    if (pair_ok<C>(V, w, ldv, p0)) {
        // two points per lane, 16-byte loads and stores
        float4* __restrict__ w4 = (float4*)(w + p0);
        const int64_t npair = (p1 - p0) >> 1;
        for (int64_t k = threadIdx.x; k < npair; k += KT) {
            const float4 a = w4[k];
            double ax = a.x, ay = a.y, bx = a.z, by = a.w;
            // unrolled so that several basis loads are in flight (same order of the sums)
#pragma unroll 8
            for (int i = 0; i < nv; ++i) {
                const float4 v = ((const float4*)(V + (int64_t)i * ldv + p0))[k];
                const double2 hi = h[i];
                ax -= (double)v.x * hi.x - (double)v.y * hi.y;
                ay -= (double)v.x * hi.y + (double)v.y * hi.x;
                bx -= (double)v.z * hi.x - (double)v.w * hi.y;
                by -= (double)v.z * hi.y + (double)v.w * hi.x;
            }
            w4[k] = float4{(float)ax, (float)ay, (float)bx, (float)by};
        }
        if (((p1 - p0) & 1) && threadIdx.x == KT - 1) {
            const int64_t p = p1 - 1;
            const C wp = w[p];
            double ax = wp.x, ay = wp.y;
#pragma unroll 8
            for (int i = 0; i < nv; ++i) {
                const C v = V[(int64_t)i * ldv + p];
                const double2 hi = h[i];
                ax -= (double)v.x * hi.x - (double)v.y * hi.y;
                ay -= (double)v.x * hi.y + (double)v.y * hi.x;
            }
            w[p] = from_d2<C>(double2{ax, ay});
        }
    } else {
        for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
            const C wp = w[p];
            double ax = wp.x, ay = wp.y;
#pragma unroll 8
            for (int i = 0; i < nv; ++i) {
                const C v = V[(int64_t)i * ldv + p];
                const double2 hi = h[i];
                ax -= (double)v.x * hi.x - (double)v.y * hi.y;
                ay -= (double)v.x * hi.y + (double)v.y * hi.x;
            }
            w[p] = from_d2<C>(double2{ax, ay});
        }
    }
}

template <typename C>
__device__ __forceinline__ void dots_body(const C* __restrict__ V, int64_t ldv, int nv, const C* __restrict__ w,
                                 int64_t p0, int64_t p1, double2* __restrict__ part) {
    if (nv > 2 * IC) {
        dots_body_waves(V, ldv, nv, w, p0, p1, part);
        return;
    }
    if constexpr (std::is_same<C, float2>::value) {
        if (pair_ok<C>(V, w, ldv, p0)) {
            dots_body_pairs(V, ldv, nv, w, p0, p1, part);
            return;
        }
    }
    for (int i0 = 0; i0 < nv; i0 += IC) {
        double ar[IC], ai[IC];
#pragma unroll
        for (int q = 0; q < IC; ++q) ar[q] = ai[q] = 0.0;
        for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
            const C wp = w[p];
#pragma unroll
            for (int q = 0; q < IC; ++q) {
                if (i0 + q < nv) {
                    const C v = V[(int64_t)(i0 + q) * ldv + p];
                    ar[q] += (double)v.x * wp.x + (double)v.y * wp.y;
                    ai[q] += (double)v.x * wp.y - (double)v.y * wp.x;
                }
            }
        }
        block_store<IC>(ar, ai, part + i0, nv - i0);
    }
}

// part[i] = sum conj(V_i) r0 and part[off1 + i] = sum conj(V_i) r1 over the block's points
// [p0, p1), i < nv, reading V once: wavefront wv takes the groups of IC vectors IC wv,
// IC (wv + 4), ... and reduces each within the wavefront.
template <typename C>
__device__ __forceinline__ void dots2_body(const C* __restrict__ V, int64_t ldv, int nv, const C* __restrict__ r0,
                                           const C* __restrict__ r1, int64_t p0, int64_t p1,
                                           double2* __restrict__ part, int off1) {
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const bool pairs = pair_ok<C>(V, r0, ldv, p0) && pair_ok<C>(r1, r1, 0, p0);
    for (int i0 = wv * IC; i0 < nv; i0 += (KT / 64) * IC) {
        double xr[IC], xi[IC], yr[IC], yi[IC];
#pragma unroll
        for (int q = 0; q < IC; ++q) xr[q] = xi[q] = yr[q] = yi[q] = 0.0;
        bool done = false;
        if constexpr (std::is_same<C, float2>::value) {
            if (pairs) {
                const int64_t npair = (p1 - p0) >> 1;
                const float4* __restrict__ a4 = (const float4*)(r0 + p0);
                const float4* __restrict__ b4 = (const float4*)(r1 + p0);
                for (int64_t k = ln; k < npair; k += 64) {
                    const float4 a = a4[k], b = b4[k];
#pragma unroll
                    for (int q = 0; q < IC; ++q) {
                        if (i0 + q < nv) {
                            const float4 v = ((const float4*)(V + (int64_t)(i0 + q) * ldv + p0))[k];
                            xr[q] += (double)v.x * a.x + (double)v.y * a.y + (double)v.z * a.z + (double)v.w * a.w;
                            xi[q] += (double)v.x * a.y - (double)v.y * a.x + (double)v.z * a.w - (double)v.w * a.z;
                            yr[q] += (double)v.x * b.x + (double)v.y * b.y + (double)v.z * b.z + (double)v.w * b.w;
                            yi[q] += (double)v.x * b.y - (double)v.y * b.x + (double)v.z * b.w - (double)v.w * b.z;
                        }
                    }
                }
                if (((p1 - p0) & 1) && ln == 63) {   // odd tail point
                    const float2 a = r0[p1 - 1], b = r1[p1 - 1];
#pragma unroll
                    for (int q = 0; q < IC; ++q)
                        if (i0 + q < nv) {
                            const float2 v = V[(int64_t)(i0 + q) * ldv + p1 - 1];
                            xr[q] += (double)v.x * a.x + (double)v.y * a.y;
                            xi[q] += (double)v.x * a.y - (double)v.y * a.x;
                            yr[q] += (double)v.x * b.x + (double)v.y * b.y;
                            yi[q] += (double)v.x * b.y - (double)v.y * b.x;
                        }
                }
                done = true;
            }
        }
        if (!done) {
            for (int64_t p = p0 + ln; p < p1; p += 64) {
                const C a = r0[p], b = r1[p];
#pragma unroll
                for (int q = 0; q < IC; ++q) {
                    if (i0 + q < nv) {
                        const C v = V[(int64_t)(i0 + q) * ldv + p];
                        xr[q] += (double)v.x * a.x + (double)v.y * a.y;
                        xi[q] += (double)v.x * a.y - (double)v.y * a.x;
                        yr[q] += (double)v.x * b.x + (double)v.y * b.y;
                        yi[q] += (double)v.x * b.y - (double)v.y * b.x;
                    }
                }
            }
        }
        wave_store8(xr, xi, part + i0, nv - i0);
        wave_store8(yr, yi, part + off1 + i0, nv - i0);
    }
}

template <typename C>
__device__ __forceinline__ void norm_body(const C* __restrict__ w, int64_t p0, int64_t p1, double2* __restrict__ out) {
    double a[1] = {0.0}, z[1] = {0.0};
    if (pair_ok<C>(w, w, 0, p0)) {
        const float4* __restrict__ w4 = (const float4*)(w + p0);
        const int64_t npair = (p1 - p0) >> 1;
        for (int64_t k = threadIdx.x; k < npair; k += KT) {
            const float4 v = w4[k];
            a[0] += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
        }
        if (((p1 - p0) & 1) && threadIdx.x == KT - 1) {
            const C v = w[p1 - 1];
            a[0] += (double)v.x * v.x + (double)v.y * v.y;
        }
    } else {
        for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
            const C wp = w[p];
            a[0] += (double)wp.x * wp.x + (double)wp.y * wp.y;
        }
    }
    block_store<1>(a, z, out, 1);
}

// sum_b part[b * ldp + i] by one block of KT threads: thread t takes b = t mod KT, then the
// wavefront sums and the KT / 64 wavefront totals are added in order (deterministic).
__device__ inline double2 block_sum_slot(const double2* __restrict__ part, int nblk, int ldp, int i) {
    __shared__ double red[KT / 64][2];
    double a = 0, b = 0;
#pragma unroll 4
    for (int q = threadIdx.x; q < nblk; q += KT) {
        const double2 v = part[(int64_t)q * ldp + i];
        a += v.x;
        b += v.y;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6][0] = a;
        red[threadIdx.x >> 6][1] = b;
    }
    __syncthreads();
    double2 r{0.0, 0.0};
#pragma unroll
    for (int w = 0; w < KT / 64; ++w) {
        r.x += red[w][0];
        r.y += red[w][1];
    }
    return r;
}

__device__ inline double sum_parts(const double2* part, int nblk, int ldp, int slot) {
    const int ln = threadIdx.x & 63;
    double a = 0;
#pragma unroll 8
    for (int q = ln; q < nblk; q += 64) a += part[(int64_t)q * ldp + slot].x;   // loads in flight together
    return wave_sum(a);
}

__device__ inline void init_state_body(SolveState* st, const double2* part, int nblk, int ldp, double tol, int m,
                                int hist_cap) {
    double nb2 = sum_parts(part, nblk, ldp, 0);
    if (threadIdx.x == 0) {
        st->bnorm = sqrt(nb2);
        st->tol = tol;
        st->m = m;
        st->stop = 0;
        st->k = 0;
        st->its = 0;
        st->cycles = 0;
        st->flags = isfinite(nb2) ? 0 : FL_NONFINITE;
        st->est = 1.0;
        st->true_rel = 1.0;
        st->hist_cap = hist_cap;
    }
}

// Cycle start: beta = ||r|| from the residual kernel's partials, convergence test
// on the true residual, g = beta e1.
__device__ inline void cycle_start_body(SolveState* st, const double* __restrict__ rpart, int nparts, double2* g, int m) {
    const int ln = threadIdx.x & 63;
    double a = 0;
    for (int q = ln; q < nparts; q += 64) a += rpart[q];
    a = wave_sum(a);
    for (int i = ln; i <= m; i += 64) g[i] = double2{0.0, 0.0};
    if (threadIdx.x == 0) {
        const double beta = sqrt(a);
        st->beta = beta;
        st->k = 0;
        st->true_rel = st->bnorm > 0 ? beta / st->bnorm : 0.0;
        int stop = 0;
        if (!isfinite(beta)) {
            st->flags |= FL_NONFINITE;
            stop = 1;
        } else if (st->true_rel <= st->tol || beta == 0.0) {
            st->flags |= FL_CONVERGED;
            stop = 1;
        } else if (st->flags & (FL_NONFINITE | FL_BREAKDOWN)) {
            stop = 1;
        }
        st->stop = stop;
        st->inv_beta = beta > 0 ? 1.0 / beta : 0.0;
        g[0] = double2{beta, 0.0};
    }
}

constexpr int AF_WIN = 128;   // rotations staged in LDS by the Hessenberg kernels

// Lane 0: apply the previous rotations to Hessenberg column jc (entries col(i), i <= jc), form
// rotation jc from the rotated diagonal entry and the subdiagonal hn, update g and the residual
// estimate, and decide whether the cycle ends (converged, breakdown against wn0 = ||w|| before
// orthogonalisation, non-finite values, history full). csl / snl hold the first AF_WIN rotations.
template <class Col>
__device__ inline void givens_tail(SolveState* st, double2* __restrict__ R, double* __restrict__ cs,
                                   double2* __restrict__ sn, double2* __restrict__ g, double* __restrict__ hist,
                                   int jc, double hn, double wn0, Col hcol, const double* csl, const double2* snl) {
    const int m = st->m;
    double2* col = R + (int64_t)jc * (m + 1);
    double2 cur = hcol(0);
    bool bad = !isfinite(hn) || !isfinite(wn0) || !isfinite(cur.x) || !isfinite(cur.y);
#pragma unroll 4
    for (int i = 0; i < jc; ++i) {   // previous rotations: (x0, x1) -> (c x0 + s x1, -conj(s) x0 + c x1)
        const double2 x1 = hcol(i + 1);
        const double c = i < AF_WIN ? csl[i] : cs[i];
        const double2 s = i < AF_WIN ? snl[i] : sn[i];
        bad |= !isfinite(x1.x) || !isfinite(x1.y);
        col[i] = cadd(double2{c * cur.x, c * cur.y}, cmul(s, x1));
        cur = csub(double2{c * x1.x, c * x1.y}, cmulc(s, cur));
    }
    if (bad) {
        st->flags |= FL_NONFINITE;
        st->stop = 1;
        return;
    }
    const double2 a = cur;
    const double aa = sqrt(a.x * a.x + a.y * a.y);
    const double rho = sqrt(aa * aa + hn * hn);
    double c;
    double2 s, r;
    if (rho == 0.0) {
        c = 1.0;
        s = double2{0.0, 0.0};
        r = double2{0.0, 0.0};
    } else if (aa == 0.0) {
        c = 0.0;
        s = double2{1.0, 0.0};   // conj(b) / |b| with b = hn real > 0
        r = double2{hn, 0.0};
    } else {
        const double2 ph = double2{a.x / aa, a.y / aa};
        c = aa / rho;
        s = double2{ph.x * hn / rho, ph.y * hn / rho};
        r = double2{ph.x * rho, ph.y * rho};
    }
    cs[jc] = c;
    sn[jc] = s;
    col[jc] = r;
    col[jc + 1] = double2{0.0, 0.0};
    const double2 gj = g[jc];
    g[jc + 1] = double2{-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x)};   // -conj(s) g_j
    g[jc] = double2{c * gj.x, c * gj.y};
    const double est = sqrt(g[jc + 1].x * g[jc + 1].x + g[jc + 1].y * g[jc + 1].y) / st->bnorm;
    st->est = est;
    if (st->its < st->hist_cap) hist[st->its] = est;
    st->its += 1;
    if (jc == 0) st->cycles += 1;
    st->k = jc + 1;
    st->wnorm0 = wn0;
    if (hn <= 1e-14 * wn0) {
        st->flags |= FL_BREAKDOWN;
        st->stop = 1;
        st->inv_h = 0.0;
        return;
    }
    st->inv_h = 1.0 / hn;
    if (est <= st->tol || st->its >= st->hist_cap) st->stop = 1;
}

// One block (every thread calls it): assemble Hessenberg column j (h1 + h2), apply the previous rotations to it,
// form rotation j, update g and the residual estimate, decide whether the cycle ends. The
// rotations run as one chain in registers on lane 0; the column entries and rotations it reads
// do not depend on its stores, so their loads can be issued ahead of the chain.
__device__ inline void arnoldi_finish_body(SolveState* st, double2* __restrict__ R, double* __restrict__ cs,
                                           double2* __restrict__ sn, double2* __restrict__ g,
                                           const double2* __restrict__ h1, const double2* __restrict__ h2,
                                           const double2* __restrict__ part, int nblk, int ldp, int j,
                                           double* __restrict__ hist) {
    const int stopped = st->stop;   // tested after the loads below (they write LDS only)
    const double hn2 = sum_parts(part, nblk, ldp, 0);     // ||w||^2 after orthogonalisation
    // stage the column and the first AF_WIN rotations in LDS with one parallel pass
    __shared__ double2 hl[AF_WIN + 1], snl[AF_WIN];
    __shared__ double csl[AF_WIN];
    for (int i = threadIdx.x; i <= j && i <= AF_WIN; i += blockDim.x) {
        double2 a = h1[i];
        if (h2) a = cadd(a, h2[i]);
        hl[i] = a;
        if (i < j && i < AF_WIN) {
            csl[i] = cs[i];
            snl[i] = sn[i];
        }
    }
    __syncthreads();
    if (stopped || threadIdx.x != 0) return;
    const double wn0 = sqrt(h1[j + 1].x);
    const double hn = sqrt(hn2);
    auto hcol = [&](int i) {
        if (i <= AF_WIN) return hl[i];
        double2 a = h1[i];
        if (h2) a = cadd(a, h2[i]);
        return a;
    };
    givens_tail(st, R, cs, sn, g, hist, j, hn, wn0, hcol, csl, snl);
}

// Delayed reorthogonalisation (one reduction per step), one block of 64 threads. At step j the
// reduction gave red[i] = conj(q_i) v~ (i < j; red[j] = ||v~||^2) and red[j + 1 + i] =
// conj(q_i) w (i < j; red[2j + 1] = conj(v~) w), red[2j + 2].x = ||w||^2, where v~ (slot j) is the
// previous step's once-projected vector and w = A z_j with z_j the network applied to v~.
// With a = red[0..j), nu = sqrt(||v~||^2 - ||a||^2) (Pythagoras):
//  * column j - 1 is complete: its pending first-pass entries plus a, subdiagonal nu (Givens
//    step, estimate, stop decisions as for the one-step form);
//  * q_j = (v~ - Q a) / nu, and the first pass of column j against [Q, q_j]: b = red[j+1 ..),
//    h_jj = (conj(v~) w - a^H b) / nu (pending entries of column j; coefficients for the update);
//  * the update pass then forms the next network input v~_{j+1} = w - Q b - h_jj q_j (its norm,
//    which sets the network's input scale, comes from that pass's partial sums: a Pythagorean
//    estimate ||w||^2 - ||b||^2 - |h_jj|^2 loses all accuracy with FP32 vectors once
//    ||v~_{j+1}|| / ||w|| falls below about 1e-3, as happens late in long cycles).
// sc[2] = ||w|| of this step, sc[3] = that of the previous step (breakdown test of column j - 1).
// tail: the cycle's last call (no new column: only column j - 1 is completed).
__device__ inline void arnoldi_lag_body(SolveState* st, double2* __restrict__ R, double* __restrict__ cs,
                                        double2* __restrict__ sn, double2* __restrict__ g,
                                        double2* __restrict__ pend, double2* __restrict__ colb,
                                        double2* __restrict__ coef, double* __restrict__ sc,
                                        const double2* __restrict__ red, int j, int tail,
                                        double* __restrict__ hist) {
    if (st->stop) return;
    const int ln = threadIdx.x & 63;
    // ||a||^2, a^H b (fixed-order wavefront sums)
    double na = 0, abr = 0, abi = 0;
    for (int i = ln; i < j; i += 64) {
        const double2 a = red[i];
        na += a.x * a.x + a.y * a.y;
        if (!tail) {
            const double2 b = red[j + 1 + i];
            abr += a.x * b.x + a.y * b.y;
            abi += a.x * b.y - a.y * b.x;
        }
    }
    na = wave_sum(na);
    abr = wave_sum(abr);
    abi = wave_sum(abi);
    // v_0 comes normalised from the cycle start (g = beta e_1 relies on it): nu = 1 there
    const double nu2 = red[j].x - na;
    const double nu = j == 0 ? 1.0 : sqrt(nu2 > 0 ? nu2 : 0.0);
    // column j - 1 = pending entries + a (entry j - 1 + 1 = nu is the subdiagonal)
    __shared__ double2 snl[AF_WIN];
    __shared__ double csl[AF_WIN];
    if (j > 0) {
        for (int i = ln; i < j; i += 64) {
            colb[i] = cadd(pend[i], red[i]);
            if (i < j - 1 && i < AF_WIN) {
                csl[i] = cs[i];
                snl[i] = sn[i];
            }
        }
    }
    __syncthreads();
    if (!tail) {
        // first pass of column j, the update's coefficients and the next input scale
        const double inv_nu = nu > 0 ? 1.0 / nu : 0.0;
        const double2 hjj{(red[2 * j + 1].x - abr) * inv_nu, (red[2 * j + 1].y - abi) * inv_nu};
        for (int i = ln; i < j; i += 64) {
            pend[i] = red[j + 1 + i];
            coef[i] = red[i];                 // q_j = (v~ - sum a_i q_i) / nu
            coef[j + i] = red[j + 1 + i];     // w' = w - sum b_i q_i - h_jj q_j
        }
        if (ln == 0) {
            pend[j] = hjj;
            coef[2 * j] = hjj;
            coef[2 * j + 1] = double2{inv_nu, 0.0};
            sc[2] = sqrt(red[2 * j + 2].x);     // ||w|| before orthogonalisation: breakdown test of column j
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (j > 0) {
        // the breakdown test of column j - 1 compares nu with ||w_{j-1}|| (kept from the previous step)
        const double wn0 = sc[3];
        auto hcol = [&](int i) { return colb[i]; };
        givens_tail(st, R, cs, sn, g, hist, j - 1, nu, wn0, hcol, csl, snl);
    }
    if (!tail) sc[3] = sc[2];
}

// y = R^{-1} g over the k completed columns (trailing zero pivots dropped).
__device__ inline void backsolve_body(SolveState* st, const double2* R, const double2* g, double2* y) {
    if (threadIdx.x != 0) return;
    const int m = st->m;
    int k = st->k;
    if (st->flags & FL_NONFINITE) k = 0;
    while (k > 0) {
        const double2 d = R[(int64_t)(k - 1) * (m + 1) + (k - 1)];
        if (d.x != 0.0 || d.y != 0.0) break;
        --k;
    }
    for (int i = k - 1; i >= 0; --i) {
        double2 acc = g[i];
        for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(R[(int64_t)l * (m + 1) + i], y[l]));
        const double2 d = R[(int64_t)i * (m + 1) + i];
        const double dd = d.x * d.x + d.y * d.y;
        y[i] = double2{(acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd};
    }
    st->k = k;   // columns used by the x update
}

}  // namespace hz
