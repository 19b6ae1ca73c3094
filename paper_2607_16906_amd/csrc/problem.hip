// Problem setup and the complex Helmholtz stencil (forward, adjoint, FP64 residual).
//
// Operator (Section 2.1, eq. (1)-(3)): five-point stretched Laplacian plus k^2.
// Along one axis, position s (node or half-node) lies d(s) = max(0, npml - s,
// s - (n_t - 1 - npml)) cells into the PML, with damping sigma(s) =
// sigma_max (d / npml)^2 (eq. (2)) and stretch gamma(s) = 1 + i sigma(s) / omega.
// The node coefficients are a+[i] = 1 / (h^2 gamma(i) gamma(i+1/2)) and
// a-[i] = 1 / (h^2 gamma(i) gamma(i-1/2)), and
//   (A u)_ij = a+x[i] u_{i+1,j} + a-x[i] u_{i-1,j} + a+y[j] u_{i,j+1} + a-y[j] u_{i,j-1}
//            + (k^2_ij - a+x[i] - a-x[i] - a+y[j] - a-y[j]) u_ij,
// with u = 0 outside the grid. A^H uses conj(a-x[i+1]) for the right neighbour,
// conj(a+x[i-1]) for the left one (likewise along y) and the conjugated diagonal.
#include <cmath>
#include <cstring>
#include <mutex>

#include "problem.h"
#include "stencil_impl.h"

namespace hz {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

// ------------------------------------------------------------------ setup kernels

__device__ inline double pml_sigma_at(double s, int nt, int npml, double smax) {
    if (npml == 0) return 0.0;
    double d = fmax(0.0, fmax((double)npml - s, s - (double)(nt - 1 - npml)));
    double r = d / (double)npml;
    return smax * r * r;
}

__device__ inline double2 cinv(double2 z) {
    double m = z.x * z.x + z.y * z.y;
    return double2{z.x / m, -z.y / m};
}

// One thread per node of one axis: forward and adjoint neighbour coefficients,
// the diagonal contribution a+[i] + a-[i], and sigma at the node.
__global__ void k_setup_axis(int nt, int npml, double h, double omega, double smax,
                             double2* fP, double2* fM, double2* aP, double2* aM, double2* dsum,
                             float2* fPf, float2* fMf, float2* aPf, float2* aMf, float2* dsumf,
                             double* sig) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    auto gam = [&](double s) { return double2{1.0, pml_sigma_at(s, nt, npml, smax) / omega}; };
    auto coef = [&](double s0, double s1) {   // 1 / (h^2 gamma(s0) gamma(s1))
        double2 g = cmul(gam(s0), gam(s1));
        return cinv(double2{g.x * h * h, g.y * h * h});
    };
    double2 ap = coef(i, i + 0.5), am = coef(i, i - 0.5);
    double2 ap_left = coef(i - 1, i - 0.5);    // a+[i-1]
    double2 am_right = coef(i + 1, i + 0.5);   // a-[i+1]
    double2 z = double2{0.0, 0.0};
    fP[i] = ap;
    fM[i] = am;
    aP[i] = (i + 1 < nt) ? cconj(am_right) : z;    // multiplies u[i+1] in A^H
    aM[i] = (i - 1 >= 0) ? cconj(ap_left) : z;     // multiplies u[i-1] in A^H
    dsum[i] = cadd(ap, am);
    fPf[i] = from_d2<float2>(fP[i]);
    fMf[i] = from_d2<float2>(fM[i]);
    aPf[i] = from_d2<float2>(aP[i]);
    aMf[i] = from_d2<float2>(aM[i]);
    dsumf[i] = from_d2<float2>(dsum[i]);
    sig[i] = pml_sigma_at(i, nt, npml, smax);
}

__global__ void k_setup_field(const float* c, int64_t n, double omega, double cref,
                              float* k2f, double* k2d, double* cnd, int* bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ci = (double)c[i];
    if (!(ci > 0.0) || !isfinite(ci)) {
        atomicOr(bad, 1);
        ci = cref;
    }
    double k = omega * cref / ci;
    k2d[i] = k * k;
    k2f[i] = (float)(k * k);
    cnd[i] = ci / cref;
}

// ------------------------------------------------------------------ stencil


template <typename T, int MODE>
__global__ __launch_bounds__(ST_THREADS) void k_stencil(
    const cplx_t<T>* __restrict__ u, cplx_t<T>* __restrict__ y, const cplx_t<T>* __restrict__ b,
    const T* __restrict__ k2, const cplx_t<T>* __restrict__ cE, const cplx_t<T>* __restrict__ cW,
    const cplx_t<T>* __restrict__ cN, const cplx_t<T>* __restrict__ cS,
    const cplx_t<T>* __restrict__ dx, const cplx_t<T>* __restrict__ dy, int conj_diag, int nx, int ny,
    double* __restrict__ part, const int* __restrict__ skip) {
    if (skip && *skip) return;
    stencil_tile<T, MODE>(u, y, b, k2, cE, cW, cN, cS, dx, dy, conj_diag, nx, ny,
                          part ? part + blockIdx.y * gridDim.x + blockIdx.x : nullptr, blockIdx.x * ST_TX,
                          blockIdx.y * ST_TY);
}

bool stencil_pairs_ok(const hz_problem* p, const void* x, const void* y) {
    return (p->nxt & 1) == 0 && ((((uintptr_t)x) | ((uintptr_t)y)) & 15) == 0;
}

__global__ __launch_bounds__(256) void k_stencil_wide(const float2* __restrict__ u, float2* __restrict__ y,
                                                      const float* __restrict__ k2, const float2* __restrict__ cE,
                                                      const float2* __restrict__ cW, const float2* __restrict__ cN,
                                                      const float2* __restrict__ cS, const float2* __restrict__ dx,
                                                      const float2* __restrict__ dy, int conj_diag, int nx, int ny,
                                                      const int* __restrict__ skip) {
    if (skip && *skip) return;
    stencil_tile_wide(u, y, k2, cE, cW, cN, cS, dx, dy, conj_diag, nx, ny, blockIdx.x * SW_TX, blockIdx.y * SW_TY);
}

StencilCoef stencil_coef(const hz_problem* p, bool fp64, bool adjoint) {
    StencilCoef c;
    if (fp64) {
        c.E = adjoint ? p->aE_d : p->fE_d;
        c.W = adjoint ? p->aW_d : p->fW_d;
        c.N = adjoint ? p->aN_d : p->fN_d;
        c.S = adjoint ? p->aS_d : p->fS_d;
        c.dx = p->dx_d;
        c.dy = p->dy_d;
        c.k2 = p->k2d;
    } else {
        c.E = adjoint ? p->aE_f : p->fE_f;
        c.W = adjoint ? p->aW_f : p->fW_f;
        c.N = adjoint ? p->aN_f : p->fN_f;
        c.S = adjoint ? p->aS_f : p->fS_f;
        c.dx = p->dx_f;
        c.dy = p->dy_f;
        c.k2 = p->k2f;
    }
    c.conj_diag = adjoint ? 1 : 0;
    return c;
}

static dim3 stencil_grid(const hz_problem* p) {
    return dim3((p->nxt + ST_TX - 1) / ST_TX, (p->nyt + ST_TY - 1) / ST_TY);
}
int stencil_blocks(const hz_problem* p) {
    if (is_spectral(p)) return spectral_blocks(p);
    dim3 g = stencil_grid(p);
    return (int)(g.x * g.y);
}

int launch_stencil(const hz_problem* p, bool fp64, bool adjoint, const void* x, void* y, hipStream_t s,
                   const int* skip) {
    if (is_spectral(p)) return launch_spectral(p, fp64, adjoint, x, y, s, skip);
    StencilCoef c = stencil_coef(p, fp64, adjoint);
    dim3 grid = stencil_grid(p);
    if (fp64) {
        hipLaunchKernelGGL((k_stencil<double, ST_PLAIN>), grid, dim3(ST_THREADS), 0, s,
                           (const double2*)x, (double2*)y, nullptr, (const double*)c.k2,
                           (const double2*)c.E, (const double2*)c.W, (const double2*)c.N, (const double2*)c.S,
                           (const double2*)c.dx, (const double2*)c.dy, c.conj_diag, p->nxt, p->nyt,
                           nullptr, skip);
    } else if (stencil_pairs_ok(p, x, y)) {
        const dim3 gw((p->nxt + SW_TX - 1) / SW_TX, (p->nyt + SW_TY - 1) / SW_TY);
        hipLaunchKernelGGL(k_stencil_wide, gw, dim3(256), 0, s, (const float2*)x, (float2*)y, (const float*)c.k2,
                           (const float2*)c.E, (const float2*)c.W, (const float2*)c.N, (const float2*)c.S,
                           (const float2*)c.dx, (const float2*)c.dy, c.conj_diag, p->nxt, p->nyt, skip);
    } else {
        hipLaunchKernelGGL((k_stencil<float, ST_PLAIN>), grid, dim3(ST_THREADS), 0, s,
                           (const float2*)x, (float2*)y, nullptr, (const float*)c.k2,
                           (const float2*)c.E, (const float2*)c.W, (const float2*)c.N, (const float2*)c.S,
                           (const float2*)c.dx, (const float2*)c.dy, c.conj_diag, p->nxt, p->nyt,
                           nullptr, skip);
    }
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_resid64(const hz_problem* p, const double2* b, const double2* x, double2* r,
                   double* part, const int* skip, hipStream_t s) {
    if (is_spectral(p)) return launch_spectral_resid64(p, b, x, r, part, skip, s);
    StencilCoef c = stencil_coef(p, true, false);
    hipLaunchKernelGGL((k_stencil<double, ST_RESID>), stencil_grid(p), dim3(ST_THREADS), 0, s,
                       x, r, b, (const double*)c.k2, (const double2*)c.E, (const double2*)c.W,
                       (const double2*)c.N, (const double2*)c.S, (const double2*)c.dx, (const double2*)c.dy,
                       0, p->nxt, p->nyt, part, skip);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

int launch_resid32(const hz_problem* p, const float2* b, const float2* x, float2* y, double* part, hipStream_t s) {
    if (is_spectral(p)) {
        set_error("the FP32 residual kernel takes the finite-difference operator only");
        return HZ_ERR_ARG;
    }
    StencilCoef c = stencil_coef(p, false, false);
    hipLaunchKernelGGL((k_stencil<float, ST_RESID>), stencil_grid(p), dim3(ST_THREADS), 0, s, x, y, b,
                       (const float*)c.k2, (const float2*)c.E, (const float2*)c.W, (const float2*)c.N,
                       (const float2*)c.S, (const float2*)c.dx, (const float2*)c.dy, 0, p->nxt, p->nyt, part,
                       (const int*)nullptr);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

}  // namespace hz

using namespace hz;

extern "C" const char* hz_last_error(void) { return g_last_error.c_str(); }

extern "C" int hz_problem_create(const hz_grid* g, const float* c_dev, void* stream, hz_problem** out) {
    clear_error();
    HZ_CHECK_ARG(g && c_dev && out, "hz_problem_create: NULL argument");
    HZ_CHECK_ARG(g->nx >= 1 && g->ny >= 1 && g->npml >= 0, "hz_problem_create: bad grid sizes");
    HZ_CHECK_ARG(g->h > 0 && g->omega > 0 && g->sigma_max >= 0 && g->c_ref > 0,
                 "hz_problem_create: h, omega, c_ref must be > 0 and sigma_max >= 0");
    HZ_CHECK_ARG(g->disc == HZ_DISC_FD || g->disc == HZ_DISC_SPECTRAL, "hz_problem_create: bad disc");
    const int nxt = g->nx + 2 * g->npml, nyt = g->ny + 2 * g->npml;
    HZ_CHECK_ARG((int64_t)nxt * nyt < (int64_t)1 << 31, "hz_problem_create: grid too large");
    HZ_CHECK_ARG(g->disc != HZ_DISC_SPECTRAL || (nxt <= 8192 && nyt <= 8192),
                 "hz_problem_create: the spectral operator takes at most 8192 nodes per axis");
    hipStream_t s = (hipStream_t)stream;
    hz_problem* p = new hz_problem();
    p->uid = next_handle_uid();
    p->g = *g;
    p->nxt = nxt;
    p->nyt = nyt;
    p->n = (int64_t)nxt * nyt;
    const int64_t n = p->n;
    Carver cv(nullptr, 0);
    auto layout = [&](Carver& c) {
        p->k2f = c.take<float>(n);
        p->k2d = c.take<double>(n);
        p->cnd = c.take<double>(n);
        double2** d1[] = {&p->fE_d, &p->fW_d, &p->aE_d, &p->aW_d, &p->dx_d};
        for (auto q : d1) *q = c.take<double2>(nxt);
        double2** d2[] = {&p->fN_d, &p->fS_d, &p->aN_d, &p->aS_d, &p->dy_d};
        for (auto q : d2) *q = c.take<double2>(nyt);
        float2** f1[] = {&p->fE_f, &p->fW_f, &p->aE_f, &p->aW_f, &p->dx_f};
        for (auto q : f1) *q = c.take<float2>(nxt);
        float2** f2[] = {&p->fN_f, &p->fS_f, &p->aN_f, &p->aS_f, &p->dy_f};
        for (auto q : f2) *q = c.take<float2>(nyt);
        p->sigx = c.take<double>(nxt);
        p->sigy = c.take<double>(nyt);
        if (g->disc == HZ_DISC_SPECTRAL) {
            p->dtx = c.take<double>(nxt);
            p->dty = c.take<double>(nyt);
            p->Mx_d = c.take<double2>((size_t)nxt * nxt);
            p->My_d = c.take<double2>((size_t)nyt * nyt);
            p->Mx_f = c.take<float2>((size_t)nxt * nxt);
            p->My_f = c.take<float2>((size_t)nyt * nyt);
        }
        return c.take<int>(1);
    };
    layout(cv);
    size_t bytes = cv.off + 256;
    if (hipMalloc(&p->block, bytes) != hipSuccess) {
        delete p;
        set_error("hz_problem_create: hipMalloc failed");
        return HZ_ERR_HIP;
    }
    Carver real(p->block, bytes);
    int* bad = layout(real);
    int rc = HZ_OK;
    int hbad = 0;
    do {
        if (hipMemsetAsync(bad, 0, sizeof(int), s) != hipSuccess) { rc = HZ_ERR_HIP; break; }
        hipLaunchKernelGGL(k_setup_axis, dim3((nxt + 127) / 128), dim3(128), 0, s, nxt, g->npml, g->h,
                           g->omega, g->sigma_max, p->fE_d, p->fW_d, p->aE_d, p->aW_d, p->dx_d, p->fE_f,
                           p->fW_f, p->aE_f, p->aW_f, p->dx_f, p->sigx);
        hipLaunchKernelGGL(k_setup_axis, dim3((nyt + 127) / 128), dim3(128), 0, s, nyt, g->npml, g->h,
                           g->omega, g->sigma_max, p->fN_d, p->fS_d, p->aN_d, p->aS_d, p->dy_d, p->fN_f,
                           p->fS_f, p->aN_f, p->aS_f, p->dy_f, p->sigy);
        hipLaunchKernelGGL(k_setup_field, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c_dev, n,
                           g->omega, g->c_ref, p->k2f, p->k2d, p->cnd, bad);
        if (hipGetLastError() != hipSuccess) { rc = HZ_ERR_HIP; break; }
        if (g->disc == HZ_DISC_SPECTRAL && spectral_setup(p, s) != HZ_OK) { rc = HZ_ERR_HIP; break; }
        if (hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) { rc = HZ_ERR_HIP; break; }
        if (hipStreamSynchronize(s) != hipSuccess) { rc = HZ_ERR_HIP; break; }
    } while (0);
    if (rc == HZ_OK && hbad) {
        rc = HZ_ERR_NONFINITE;
        set_error("hz_problem_create: velocity must be finite and > 0 everywhere");
    } else if (rc != HZ_OK) {
        set_error("hz_problem_create: HIP error during setup");
    }
    if (rc != HZ_OK) {
        (void)hipFree(p->block);
        delete p;
        return rc;
    }
    *out = p;
    return HZ_OK;
}

extern "C" int hz_problem_destroy(hz_problem* p) {
    clear_error();
    if (!p) return HZ_OK;
    fgmres_graph_cache_evict(p->uid);
    HZ_HIP(hipFree(p->block));
    delete p;
    return HZ_OK;
}

extern "C" int hz_problem_dims(const hz_problem* p, int64_t* n, int32_t* nxt, int32_t* nyt) {
    clear_error();
    HZ_CHECK_ARG(p, "hz_problem_dims: NULL problem");
    if (n) *n = p->n;
    if (nxt) *nxt = p->nxt;
    if (nyt) *nyt = p->nyt;
    return HZ_OK;
}

extern "C" int hz_op_apply(const hz_problem* p, hz_dtype dtype, int adjoint, const void* x, void* y,
                           void* stream) {
    clear_error();
    HZ_CHECK_ARG(p && x && y, "hz_op_apply: NULL argument");
    HZ_CHECK_ARG(dtype == HZ_C64 || dtype == HZ_C128, "hz_op_apply: dtype must be HZ_C64 or HZ_C128");
    HZ_CHECK_ARG(x != y, "hz_op_apply: x and y must not overlap");
    return launch_stencil(p, dtype == HZ_C128, adjoint != 0, x, y, (hipStream_t)stream);
}
