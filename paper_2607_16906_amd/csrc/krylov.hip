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
#include <cmath>

#include "krylov.h"

namespace hz {

constexpr int KT = 256;   // threads per block of the vector kernels
constexpr int IC = 8;     // inner products accumulated per sweep

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

// Sum NV pairs over the block and store them as part[slot0 + q] (thread 0 .. writes).
template <int NV>
__device__ inline void block_store(double (&ar)[NV], double (&ai)[NV], double2* out, int cnt) {
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

template <typename C>
__device__ inline void dots_body(const C* __restrict__ V, int64_t ldv, int nv, const C* __restrict__ w,
                                 int64_t p0, int64_t p1, double2* __restrict__ part) {
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

template <typename C>
__device__ inline void norm_body(const C* __restrict__ w, int64_t p0, int64_t p1, double2* __restrict__ out) {
    double a[1] = {0.0}, z[1] = {0.0};
    for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
        const C wp = w[p];
        a[0] += (double)wp.x * wp.x + (double)wp.y * wp.y;
    }
    block_store<1>(a, z, out, 1);
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

template <typename C, int MODE>
__global__ __launch_bounds__(KT) void k_update(const C* __restrict__ V, int64_t ldv, int nv,
                                               const double2* __restrict__ h, C* __restrict__ w, int64_t n,
                                               int64_t per, double2* __restrict__ part, int ldp,
                                               const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int64_t p0 = blockIdx.x * per, p1 = min(n, p0 + per);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += KT) {
        const C wp = w[p];
        double ax = wp.x, ay = wp.y;
        for (int i = 0; i < nv; ++i) {
            const C v = V[(int64_t)i * ldv + p];
            const double2 hi = h[i];
            ax -= (double)v.x * hi.x - (double)v.y * hi.y;
            ay -= (double)v.x * hi.y + (double)v.y * hi.x;
        }
        w[p] = from_d2<C>(double2{ax, ay});
    }
    // each thread reads back only the points it wrote: no barrier needed before the sweeps
    double2* mine = part + (int64_t)blockIdx.x * ldp;
    if (MODE == 1) dots_body(V, ldv, nv, w, p0, p1, mine);
    if (MODE == 2) norm_body(w, p0, p1, mine);
}

__global__ __launch_bounds__(KT) void k_finalize(const double2* __restrict__ part, int nblk, int ldp, int cnt,
                                                 double2* __restrict__ out, const int* __restrict__ skip) {
    if (skip && *skip) return;
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    for (int i = wv; i < cnt; i += KT / 64) {
        double a = 0, b = 0;
        for (int q = ln; q < nblk; q += 64) {
            const double2 v = part[(int64_t)q * ldp + i];
            a += v.x;
            b += v.y;
        }
        a = wave_sum(a);
        b = wave_sum(b);
        if (ln == 0) out[i] = double2{a, b};
    }
}

__device__ inline double sum_parts(const double2* part, int nblk, int ldp, int slot) {
    const int ln = threadIdx.x & 63;
    double a = 0;
    for (int q = ln; q < nblk; q += 64) a += part[(int64_t)q * ldp + slot].x;
    return wave_sum(a);
}

// ||b|| from the partials in slot 0; resets the counters.
__global__ void k_init_state(SolveState* st, const double2* part, int nblk, int ldp, double tol, int m,
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
__global__ void k_cycle_start(SolveState* st, const double* __restrict__ rpart, int nparts, double2* g, int m) {
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

// One wavefront: assemble Hessenberg column j, rotate it, form rotation j,
// update g and the residual estimate, decide whether the cycle ends.
__global__ void k_arnoldi_finish(SolveState* st, double2* R, double* cs, double2* sn, double2* g,
                                 const double2* h1, const double2* h2, const double2* part, int nblk, int ldp,
                                 int j, double* hist) {
    if (st->stop) return;
    const int m = st->m;
    const int ln = threadIdx.x & 63;
    const double hn2 = sum_parts(part, nblk, ldp, 0);     // ||w||^2 after orthogonalisation
    double2* col = R + (int64_t)j * (m + 1);
    for (int i = ln; i <= j; i += 64) {
        double2 a = h1[i];
        if (h2) a = cadd(a, h2[i]);
        col[i] = a;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double wn0 = sqrt(h1[j + 1].x);
    const double hn = sqrt(hn2);
    bool bad = !isfinite(hn) || !isfinite(wn0);
    for (int i = 0; i <= j; ++i) bad |= !isfinite(col[i].x) || !isfinite(col[i].y);
    if (bad) {
        st->flags |= FL_NONFINITE;
        st->stop = 1;
        return;
    }
    for (int i = 0; i < j; ++i) {   // previous rotations
        const double c = cs[i];
        const double2 s = sn[i];
        const double2 x0 = col[i], x1 = col[i + 1];
        col[i] = cadd(double2{c * x0.x, c * x0.y}, cmul(s, x1));
        col[i + 1] = csub(double2{c * x1.x, c * x1.y}, cmulc(s, x0));   // -conj(s) x0 + c x1
    }
    const double2 a = col[j];
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
    cs[j] = c;
    sn[j] = s;
    col[j] = r;
    col[j + 1] = double2{0.0, 0.0};
    const double2 gj = g[j];
    g[j + 1] = double2{-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x)};   // -conj(s) g_j
    g[j] = double2{c * gj.x, c * gj.y};
    const double est = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y) / st->bnorm;
    st->est = est;
    if (st->its < st->hist_cap) hist[st->its] = est;
    st->its += 1;
    if (j == 0) st->cycles += 1;
    st->k = j + 1;
    st->wnorm0 = wn0;
    if (hn <= 1e-14 * wn0) {
        st->flags |= FL_BREAKDOWN;
        st->stop = 1;
        st->inv_h = 0.0;
        return;
    }
    st->inv_h = 1.0 / hn;
    if (est <= st->tol) st->stop = 1;
}

// y = R^{-1} g over the k completed columns (trailing zero pivots dropped).
__global__ void k_backsolve(SolveState* st, const double2* R, const double2* g, double2* y) {
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
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(KT), 0, s, part, nblk, ldp, cnt, out, skip);
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
        if (mode == 0) HZ_UPD(float2, 0);
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
