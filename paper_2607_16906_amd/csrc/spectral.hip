// Fourier-differentiation (pseudo-spectral) form of the Helmholtz operator with PML: the
// discretization of Section 2.1 / Table 1, derivatives over the whole grid taken as periodic.
//
// Per axis the spectral first derivative is the circulant matrix D[j][l] = d[(j - l) mod N] with
// d[0] = 0 and, for m != 0, d[m] = (pi / L) (-1)^m cot(pi m / N) (N even; the Nyquist mode's
// derivative vanishes at the nodes) or (pi / L) (-1)^m csc(pi m / N) (N odd), L = N h. With the
// stretching G = diag(1 / gamma), gamma = 1 + i sigma / omega at the nodes, the operator is
//     A u = u Mx^T + My u + k^2 u,   M = G D G D   (u as an [ny][nx] matrix),
// and A^H w = w conj(Mx) + My^H w + k^2 w. The library forms Mx and My once per problem
// (FP64 and FP32), so that one launch applies A: for the grids of this method (N up to a few
// thousand) the two per-axis contractions are dense complex GEMMs of 8 N FLOP per node each, run
// on the matrix cores, with no temporaries and no FFT passes.
#include "problem.h"

namespace hz {

// the circulant's first column: d[m], m = 0..n-1
__global__ void k_spec_table(double* d, int n, double h) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    if (m == 0) {
        d[0] = 0.0;
        return;
    }
    const double t = M_PI * m / n;
    const double f = (n % 2 == 0) ? cos(t) / sin(t) : 1.0 / sin(t);
    d[m] = (M_PI / (n * h)) * ((m & 1) ? -1.0 : 1.0) * f;
}

__device__ inline double2 inv_gamma(int i, int n, int npml, double omega, double sigma_max) {
    double sig = 0.0;
    if (npml > 0) {
        const double dep = fmax(0.0, fmax((double)(npml - i), (double)(i - (n - 1 - npml))));
        sig = sigma_max * (dep / npml) * (dep / npml);
    }
    // 1 / (1 + i s) = (1 - i s) / (1 + s^2), s = sigma / omega
    const double s = sig / omega;
    const double den = 1.0 + s * s;
    return double2{1.0 / den, -s / den};
}

// M[j][l] = g_j sum_k d[(j - k) mod n] g_k d[(k - l) mod n] (FP64), and its FP32 copy
__global__ void k_spec_mmat(double2* __restrict__ Md, float2* __restrict__ Mf, const double* __restrict__ d,
                            int n, int npml, double omega, double sigma_max) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (l >= n) return;
    double ar = 0.0, ai = 0.0;
    for (int k = 0; k < n; ++k) {
        const double dj = d[(j - k + n) % n];
        const double dl = d[(k - l + n) % n];
        const double2 gk = inv_gamma(k, n, npml, omega, sigma_max);
        const double c = dj * dl;
        ar += c * gk.x;
        ai += c * gk.y;
    }
    const double2 gj = inv_gamma(j, n, npml, omega, sigma_max);
    const double2 m{gj.x * ar - gj.y * ai, gj.x * ai + gj.y * ar};
    Md[(int64_t)j * n + l] = m;
    Mf[(int64_t)j * n + l] = float2{(float)m.x, (float)m.y};
}

// Matrix-core form. The two per-axis contractions are complex GEMMs, each taken as four real
// 16 x 16 x 4 MFMA products per k-step (re += a.re b.re - a.im b.im, im += a.re b.im + a.im b.re,
// the negated a.im staged beside a.im). A block of 8 wavefronts owns a 32 x 32 output tile:
// wavefronts 0-3 form the x part sum_k u[y][k] Mx'[x][k] of one 16 x 16 quarter each, wavefronts
// 4-7 the y part sum_k My'[y][k] u[k][x] of the same quarters, both over chunks of SPK k values
// staged together in LDS (the next chunk's values in registers meanwhile). The y part is then
// added to the x part (in that order) and the epilogue adds k^2 u; for RESID it forms
// r = b - A u with the tile's ||r||^2 in part[tile]. Mx' = Mx and My' = My, or for ADJ
// Mx'[x][k] = conj(Mx[k][x]) and My'[y][k] = conj(My[k][y]). FP32 takes v_mfma_f32_16x16x4_f32,
// FP64 v_mfma_f64_16x16x4_f64.
constexpr int SPT = 32;     // output tile edge
constexpr int SPK = 16;     // k values per chunk
constexpr int SPW = 512;    // threads per block

template <typename T>
struct SpecMma;
template <>
struct SpecMma<float> {
    typedef __attribute__((ext_vector_type(4))) float V;
    __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row_of(int lg, int r) { return 4 * lg + r; }
};
template <>
struct SpecMma<double> {
    typedef __attribute__((ext_vector_type(4))) double V;
    __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row_of(int lg, int r) { return lg + 4 * r; }
};

template <typename C, bool ADJ, bool RESID>
__global__ __launch_bounds__(SPW) void k_spectral(const C* __restrict__ u, C* __restrict__ y, const C* __restrict__ b,
                                                  const C* __restrict__ Mx, const C* __restrict__ My,
                                                  const decltype(C{}.x)* __restrict__ k2, int nx, int ny,
                                                  double* __restrict__ part, const int* __restrict__ skip) {
    using T = decltype(C{}.x);
    using M = SpecMma<T>;
    using V = typename M::V;
    if (skip && *skip) return;
    // [row][k] operands (u rows for x, My' rows for y) and [k][col] operands (Mx' for x, u for y),
    // as real and imaginary planes, one padding element per row
    __shared__ T sa[2][2][SPT][SPK + 1];   // [part][re/im][row][k]
    __shared__ T sb[2][2][SPK][SPT + 1];   // [part][re/im][k][col]
    __shared__ V sy[4][2][64];            // y-part accumulators handed to the x-part wavefronts
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int prt = wv >> 2;              // 0: x part, 1: y part
    const int q = wv & 3;                 // output quarter: rows 16 (q / 2), columns 16 (q % 2)
    const int lr = lane & 15, lg = lane >> 4;
    const int x0 = blockIdx.x * SPT, y0 = blockIdx.y * SPT;
    const int nch = (max(nx, ny) + SPK - 1) / SPK;
    // staging: each thread moves one [row][k] and one [k][col] element of each part per chunk
    // (1024 + 1024 elements, 512 threads, two of each kind per thread)
    C ra[2][2], rb[2][2];
    auto gload = [&](int ch) {
        const int k0 = ch * SPK;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = threadIdx.x + SPW * i;          // 0 .. 1023
            const int pp = e >> 9, f = e & 511;           // part, element of the 32 x 16 / 16 x 32 tile
            if (pp == 0) {
                // x part: a = u[y0 + r][k0 + kk] (k fastest); b = Mx'[x0 + c][k0 + kk]
                const int r = f / SPK, kk = f % SPK;
                const int gy = y0 + r, gk = k0 + kk;
                ra[i][0] = (gy < ny && gk < nx) ? u[(int64_t)gy * nx + gk] : C{0, 0};
                if (ADJ) {   // conj(Mx[k][x]): x fastest
                    const int kr = f / SPT, c = f % SPT;
                    const int gx = x0 + c, gk2 = k0 + kr;
                    const C v = (gx < nx && gk2 < nx) ? Mx[(int64_t)gk2 * nx + gx] : C{0, 0};
                    rb[i][0] = C{v.x, -v.y};
                } else {     // Mx[x][k]: k fastest
                    const int c = f / SPK, kk2 = f % SPK;
                    const int gx = x0 + c, gk2 = k0 + kk2;
                    rb[i][0] = (gx < nx && gk2 < nx) ? Mx[(int64_t)gx * nx + gk2] : C{0, 0};
                }
            } else {
                // y part: a = My'[y0 + r][k0 + kk]; b = u[k0 + kk][x0 + c] (x fastest)
                if (ADJ) {   // conj(My[k][y]): y fastest
                    const int kk = f / SPT, r = f % SPT;
                    const int gy = y0 + r, gk = k0 + kk;
                    const C v = (gy < ny && gk < ny) ? My[(int64_t)gk * ny + gy] : C{0, 0};
                    ra[i][1] = C{v.x, -v.y};
                } else {     // My[y][k]: k fastest
                    const int r = f / SPK, kk = f % SPK;
                    const int gy = y0 + r, gk = k0 + kk;
                    ra[i][1] = (gy < ny && gk < ny) ? My[(int64_t)gy * ny + gk] : C{0, 0};
                }
                const int kr = f / SPT, c = f % SPT;
                const int gk2 = k0 + kr, gx = x0 + c;
                rb[i][1] = (gk2 < ny && gx < nx) ? u[(int64_t)gk2 * nx + gx] : C{0, 0};
            }
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int e = threadIdx.x + SPW * i;
            const int pp = e >> 9, f = e & 511;
            if (pp == 0) {
                const int r = f / SPK, kk = f % SPK;
                sa[0][0][r][kk] = ra[i][0].x;
                sa[0][1][r][kk] = ra[i][0].y;
                int kr, c;
                if (ADJ) { kr = f / SPT; c = f % SPT; } else { c = f / SPK; kr = f % SPK; }
                sb[0][0][kr][c] = rb[i][0].x;
                sb[0][1][kr][c] = rb[i][0].y;
            } else {
                int r, kk;
                if (ADJ) { kk = f / SPT; r = f % SPT; } else { r = f / SPK; kk = f % SPK; }
                sa[1][0][r][kk] = ra[i][1].x;
                sa[1][1][r][kk] = ra[i][1].y;
                const int kr = f / SPT, c = f % SPT;
                sb[1][0][kr][c] = rb[i][1].x;
                sb[1][1][kr][c] = rb[i][1].y;
            }
        }
    };
    V are, aim;
#pragma unroll
    for (int r = 0; r < 4; ++r) are[r] = aim[r] = T(0);
    const int ar0 = 16 * (q >> 1), bc0 = 16 * (q & 1);
    gload(0);
    for (int ch = 0; ch < nch; ++ch) {
        __syncthreads();
        lstore();
        __syncthreads();
        if (ch + 1 < nch) gload(ch + 1);
#pragma unroll
        for (int st = 0; st < SPK / 4; ++st) {
            const int kk = 4 * st + lg;
            const T a_re = sa[prt][0][ar0 + lr][kk], a_im = sa[prt][1][ar0 + lr][kk];
            const T b_re = sb[prt][0][kk][bc0 + lr], b_im = sb[prt][1][kk][bc0 + lr];
            are = M::mma(a_re, b_re, are);
            are = M::mma(-a_im, b_im, are);
            aim = M::mma(a_re, b_im, aim);
            aim = M::mma(a_im, b_re, aim);
        }
    }
    // y part into LDS, then the x-part wavefronts add it and finish
    if (prt == 1) {
        sy[q][0][lane] = are;
        sy[q][1][lane] = aim;
    }
    __syncthreads();
    double nrm = 0.0;
    if (prt == 0) {
        const V yre = sy[q][0][lane], yim = sy[q][1][lane];
        const int gx = x0 + bc0 + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gy = y0 + ar0 + M::row_of(lg, r);
            if (gy < ny && gx < nx) {
                const int64_t idx = (int64_t)gy * nx + gx;
                const C uq = u[idx];
                const T kq = k2[idx];
                T vr = (are[r] + yre[r]) + kq * uq.x, vi = (aim[r] + yim[r]) + kq * uq.y;
                if (RESID) {
                    vr = b[idx].x - vr;
                    vi = b[idx].y - vi;
                    nrm += (double)vr * vr + (double)vi * vi;
                }
                y[idx] = C{vr, vi};
            }
        }
    }
    if (RESID) {
        __shared__ double red[SPW / 64];
        double t = nrm;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if (lane == 0) red[wv] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double acc = 0.0;
#pragma unroll
            for (int w = 0; w < 4; ++w) acc += red[w];   // the x-part wavefronts hold the values
            part[blockIdx.y * gridDim.x + blockIdx.x] = acc;
        }
    }
}

static dim3 spectral_grid(const hz_problem* p) {
    return dim3((p->nxt + SPT - 1) / SPT, (p->nyt + SPT - 1) / SPT);
}

int spectral_blocks(const hz_problem* p) {
    const dim3 g = spectral_grid(p);
    return (int)(g.x * g.y);
}

int spectral_setup(hz_problem* p, hipStream_t s) {
    const hz_grid& g = p->g;
    hipLaunchKernelGGL(k_spec_table, dim3((p->nxt + 127) / 128), dim3(128), 0, s, p->dtx, p->nxt, g.h);
    hipLaunchKernelGGL(k_spec_table, dim3((p->nyt + 127) / 128), dim3(128), 0, s, p->dty, p->nyt, g.h);
    hipLaunchKernelGGL(k_spec_mmat, dim3((p->nxt + 127) / 128, p->nxt), dim3(128), 0, s, p->Mx_d, p->Mx_f, p->dtx,
                       p->nxt, g.npml, g.omega, g.sigma_max);
    hipLaunchKernelGGL(k_spec_mmat, dim3((p->nyt + 127) / 128, p->nyt), dim3(128), 0, s, p->My_d, p->My_f, p->dty,
                       p->nyt, g.npml, g.omega, g.sigma_max);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_spectral(const hz_problem* p, bool fp64, bool adjoint, const void* x, void* y, hipStream_t s,
                    const int* skip) {
    const dim3 grid = spectral_grid(p);
#define HZ_SP(C, A, MX, MY, K2)                                                                                  \
    hipLaunchKernelGGL((k_spectral<C, A, false>), grid, dim3(SPW), 0, s, (const C*)x, (C*)y, (const C*)nullptr, \
                       (const C*)MX, (const C*)MY, K2, p->nxt, p->nyt, (double*)nullptr, skip)
    if (fp64) {
        if (adjoint) HZ_SP(double2, true, p->Mx_d, p->My_d, p->k2d);
        else HZ_SP(double2, false, p->Mx_d, p->My_d, p->k2d);
    } else {
        if (adjoint) HZ_SP(float2, true, p->Mx_f, p->My_f, p->k2f);
        else HZ_SP(float2, false, p->Mx_f, p->My_f, p->k2f);
    }
#undef HZ_SP
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_spectral_resid32(const hz_problem* p, const float2* b, const float2* x, float2* r, double* part,
                            const int* skip, hipStream_t s) {
    hipLaunchKernelGGL((k_spectral<float2, false, true>), spectral_grid(p), dim3(SPW), 0, s, x, r, b,
                       (const float2*)p->Mx_f, (const float2*)p->My_f, p->k2f, p->nxt, p->nyt, part, skip);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_spectral_resid64(const hz_problem* p, const double2* b, const double2* x, double2* r, double* part,
                            const int* skip, hipStream_t s) {
    hipLaunchKernelGGL((k_spectral<double2, false, true>), spectral_grid(p), dim3(SPW), 0, s, x, r, b,
                       (const double2*)p->Mx_d, (const double2*)p->My_d, p->k2d, p->nxt, p->nyt, part, skip);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

}  // namespace hz
