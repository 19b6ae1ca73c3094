// Fourier-differentiation (pseudo-spectral) form of the Helmholtz operator with PML: the
// discretization of Section 2.1 / Table 1, derivatives over the whole grid taken as periodic.
//
// Per axis the spectral first derivative is the circulant matrix D[j][l] = d[(j - l) mod N] with
// d[0] = 0 and, for m != 0, d[m] = (pi / L) (-1)^m cot(pi m / N) (N even; the Nyquist mode's
// derivative vanishes at the nodes) or (pi / L) (-1)^m csc(pi m / N) (N odd), L = N h. With the
// stretching G = diag(1 / gamma), gamma = 1 + i sigma / omega at the nodes, the operator is
//     A u = u Mx^T + My u + k^2 u,   M = G D G D   (u as an [ny][nx] matrix),
// and A^H w = w conj(Mx) + My^H w + k^2 w. The library forms Mx and My once per problem
// (FP64 and FP32), so that one launch applies A: for the small grids of this method (N <= a few
// thousand) the dense per-axis contraction costs 8 N FLOP per node and reads the grid once,
// with no temporaries and no FFT passes.
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

constexpr int SP_K = 32;    // contraction chunk and tile width (x)
constexpr int SP_Y = 8;     // tile height (y)

// One SP_Y x SP_K output tile (rows y0.., columns x0..) per block of 256 threads, one output per
// thread: acc = sum_k u[y][k] Mx'[x][k] + sum_k My'[y][k] u[k][x], with Mx'[x][k] = Mx[x][k] and
// My'[y][k] = My[y][k] (ADJ: conj(Mx[k][x]), conj(My[k][y])), the x part's chunks first, then the
// y part's, each chunk staged in LDS while the next one is loaded into registers. Then
// y = acc + k^2 u, or for RESID r = b - (acc + k^2 u) with the tile's ||r||^2 in part[tile].
// Small tiles keep many blocks in flight: the grids of this method are a few hundred nodes wide.
template <typename C, bool ADJ, bool RESID>
__global__ __launch_bounds__(256) void k_spectral(const C* __restrict__ u, C* __restrict__ y, const C* __restrict__ b,
                                                  const C* __restrict__ Mx, const C* __restrict__ My,
                                                  const decltype(C{}.x)* __restrict__ k2, int nx, int ny,
                                                  double* __restrict__ part, const int* __restrict__ skip) {
    using T = decltype(C{}.x);
    if (skip && *skip) return;
    __shared__ C sa[SP_Y][SP_K + 1];     // x part: u rows; y part: My' rows
    __shared__ C sb[SP_K][SP_K + 1];     // x part: Mx' rows (sb[x][k]); y part: u (sb[k][x])
    const int tx = threadIdx.x & (SP_K - 1), ty = threadIdx.x / SP_K;
    const int x0 = blockIdx.x * SP_K, y0 = blockIdx.y * SP_Y;
    T ar = 0, ai = 0;
    auto mat = [&](const C* M, int n, int r, int k) -> C {   // M'[r][k]
        if (ADJ) {
            const C v = M[(int64_t)k * n + r];
            return C{v.x, -v.y};
        }
        return M[(int64_t)r * n + k];
    };
    constexpr int PB = SP_K * SP_K / 256;    // sb elements per thread (sa: one)
    const int ncx = (nx + SP_K - 1) / SP_K, ncy = (ny + SP_K - 1) / SP_K;
    const int nch = ncx + ncy;
    C ra, rb[PB];
    auto gload = [&](int ch) {
        const bool xp = ch < ncx;
        const int k0 = (xp ? ch : ch - ncx) * SP_K;
        {
            const int gy = y0 + ty, gk = k0 + tx;
            if (xp) ra = (gy < ny && gk < nx) ? u[(int64_t)gy * nx + gk] : C{0, 0};
            else ra = (gy < ny && gk < ny) ? mat(My, ny, gy, gk) : C{0, 0};
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int e = threadIdx.x + 256 * i;
            const int r = e / SP_K, cc = e % SP_K;
            if (xp) {
                const int gx = x0 + r, gk = k0 + cc;
                rb[i] = (gx < nx && gk < nx) ? mat(Mx, nx, gx, gk) : C{0, 0};
            } else {
                const int gk = k0 + r, gx = x0 + cc;
                rb[i] = (gk < ny && gx < nx) ? u[(int64_t)gk * nx + gx] : C{0, 0};
            }
        }
    };
    gload(0);
    for (int ch = 0; ch < nch; ++ch) {
        __syncthreads();
        sa[ty][tx] = ra;
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int e = threadIdx.x + 256 * i;
            sb[e / SP_K][e % SP_K] = rb[i];
        }
        __syncthreads();
        if (ch + 1 < nch) gload(ch + 1);
        if (ch < ncx) {
#pragma unroll 8
            for (int kk = 0; kk < SP_K; ++kk) {
                const C a = sa[ty][kk], m = sb[tx][kk];
                ar += a.x * m.x - a.y * m.y;
                ai += a.x * m.y + a.y * m.x;
            }
        } else {
#pragma unroll 8
            for (int kk = 0; kk < SP_K; ++kk) {
                const C m = sa[ty][kk], v = sb[kk][tx];
                ar += m.x * v.x - m.y * v.y;
                ai += m.x * v.y + m.y * v.x;
            }
        }
    }
    double nrm = 0.0;
    const int gy = y0 + ty, gx = x0 + tx;
    if (gy < ny && gx < nx) {
        const int64_t q = (int64_t)gy * nx + gx;
        const C uq = u[q];
        const T kk = k2[q];
        T vr = ar + kk * uq.x, vi = ai + kk * uq.y;
        if (RESID) {
            vr = b[q].x - vr;
            vi = b[q].y - vi;
            nrm = (double)vr * vr + (double)vi * vi;
        }
        y[q] = C{vr, vi};
    }
    if (RESID) {
        __shared__ double red[4];
        double t = nrm;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

constexpr int SP_B = 32;    // tile edge of the register-tiled form for large grids

// Large grids: one 32 x 32 tile per block, 2 x 2 outputs per thread (each LDS value feeds two
// products), the same chunk sequence and prefetch as k_spectral and the same summation order.
template <typename C, bool ADJ, bool RESID>
__global__ __launch_bounds__(256) void k_spectral_big(const C* __restrict__ u, C* __restrict__ y,
                                                      const C* __restrict__ b, const C* __restrict__ Mx,
                                                      const C* __restrict__ My,
                                                      const decltype(C{}.x)* __restrict__ k2, int nx, int ny,
                                                      double* __restrict__ part, const int* __restrict__ skip) {
    using T = decltype(C{}.x);
    if (skip && *skip) return;
    __shared__ C sa[SP_B][SP_B + 1];
    __shared__ C sb[SP_B][SP_B + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int x0 = blockIdx.x * SP_B, y0 = blockIdx.y * SP_B;
    T ar[2][2], ai[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) ar[a][c] = ai[a][c] = T(0);
    auto mat = [&](const C* M, int n, int r, int k) -> C {   // M'[r][k]
        if (ADJ) {
            const C v = M[(int64_t)k * n + r];
            return C{v.x, -v.y};
        }
        return M[(int64_t)r * n + k];
    };
    constexpr int PER = SP_B * SP_B / 256;
    const int ncx = (nx + SP_B - 1) / SP_B, ncy = (ny + SP_B - 1) / SP_B;
    const int nch = ncx + ncy;
    C ra[PER], rb[PER];
    auto gload = [&](int ch) {
        const bool xp = ch < ncx;
        const int k0 = (xp ? ch : ch - ncx) * SP_B;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + 256 * i;
            const int r = e / SP_B, kk = e % SP_B;
            if (xp) {
                const int gy = y0 + r, gx = x0 + r, gk = k0 + kk;
                ra[i] = (gy < ny && gk < nx) ? u[(int64_t)gy * nx + gk] : C{0, 0};
                rb[i] = (gx < nx && gk < nx) ? mat(Mx, nx, gx, gk) : C{0, 0};
            } else {
                const int gy = y0 + r, gk = k0 + kk;
                ra[i] = (gy < ny && gk < ny) ? mat(My, ny, gy, gk) : C{0, 0};
                const int gk2 = k0 + r, gx = x0 + kk;
                rb[i] = (gk2 < ny && gx < nx) ? u[(int64_t)gk2 * nx + gx] : C{0, 0};
            }
        }
    };
    gload(0);
    for (int ch = 0; ch < nch; ++ch) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + 256 * i;
            sa[e / SP_B][e % SP_B] = ra[i];
            sb[e / SP_B][e % SP_B] = rb[i];
        }
        __syncthreads();
        if (ch + 1 < nch) gload(ch + 1);
        if (ch < ncx) {
#pragma unroll 8
            for (int kk = 0; kk < SP_B; ++kk) {
                const C uu[2] = {sa[ty][kk], sa[ty + 16][kk]};
                const C mm[2] = {sb[tx][kk], sb[tx + 16][kk]};
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        ar[a][c] += uu[a].x * mm[c].x - uu[a].y * mm[c].y;
                        ai[a][c] += uu[a].x * mm[c].y + uu[a].y * mm[c].x;
                    }
            }
        } else {
#pragma unroll 8
            for (int kk = 0; kk < SP_B; ++kk) {
                const C mm[2] = {sa[ty][kk], sa[ty + 16][kk]};
                const C vv[2] = {sb[kk][tx], sb[kk][tx + 16]};
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        ar[a][c] += mm[a].x * vv[c].x - mm[a].y * vv[c].y;
                        ai[a][c] += mm[a].x * vv[c].y + mm[a].y * vv[c].x;
                    }
            }
        }
    }
    double nrm = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int gy = y0 + ty + 16 * a, gx = x0 + tx + 16 * c;
            if (gy < ny && gx < nx) {
                const int64_t q = (int64_t)gy * nx + gx;
                const C uq = u[q];
                const T kk = k2[q];
                T vr = ar[a][c] + kk * uq.x, vi = ai[a][c] + kk * uq.y;
                if (RESID) {
                    vr = b[q].x - vr;
                    vi = b[q].y - vi;
                    nrm += (double)vr * vr + (double)vi * vi;
                }
                y[q] = C{vr, vi};
            }
        }
    if (RESID) {
        __shared__ double red[4];
        double t = nrm;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

// the register-tiled form once the small tiles would exceed about 4 blocks per CU
static bool spectral_big(const hz_problem* p) {
    return (int64_t)((p->nxt + SP_K - 1) / SP_K) * ((p->nyt + SP_Y - 1) / SP_Y) > 1024;
}

static dim3 spectral_grid(const hz_problem* p) {
    if (spectral_big(p)) return dim3((p->nxt + SP_B - 1) / SP_B, (p->nyt + SP_B - 1) / SP_B);
    return dim3((p->nxt + SP_K - 1) / SP_K, (p->nyt + SP_Y - 1) / SP_Y);
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
#define HZ_SP(C, A, MX, MY, K2)                                                                                \
    if (spectral_big(p))                                                                                       \
        hipLaunchKernelGGL((k_spectral_big<C, A, false>), grid, dim3(256), 0, s, (const C*)x, (C*)y,             \
                           (const C*)nullptr, (const C*)MX, (const C*)MY, K2, p->nxt, p->nyt, (double*)nullptr, \
                           skip);                                                                              \
    else                                                                                                       \
        hipLaunchKernelGGL((k_spectral<C, A, false>), grid, dim3(256), 0, s, (const C*)x, (C*)y,                 \
                           (const C*)nullptr, (const C*)MX, (const C*)MY, K2, p->nxt, p->nyt, (double*)nullptr, \
                           skip)
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

int launch_spectral_resid64(const hz_problem* p, const double2* b, const double2* x, double2* r, double* part,
                            const int* skip, hipStream_t s) {
    if (spectral_big(p))
        hipLaunchKernelGGL((k_spectral_big<double2, false, true>), spectral_grid(p), dim3(256), 0, s, x, r, b,
                           (const double2*)p->Mx_d, (const double2*)p->My_d, p->k2d, p->nxt, p->nyt, part, skip);
    else
        hipLaunchKernelGGL((k_spectral<double2, false, true>), spectral_grid(p), dim3(256), 0, s, x, r, b,
                           (const double2*)p->Mx_d, (const double2*)p->My_d, p->k2d, p->nxt, p->nyt, part, skip);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

}  // namespace hz
