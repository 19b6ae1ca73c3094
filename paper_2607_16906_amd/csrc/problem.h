// Internal view of a problem handle and the operator kernels' launchers.
#pragma once

#include "common.h"

struct hz_problem {
    hz_grid g;
    int nxt, nyt;     // totals including the PML
    int64_t n;        // nxt * nyt
    // per-node fields
    float* k2f;       // k^2, FP32 [n]
    double* k2d;      // k^2, FP64 [n]
    double* cnd;      // c / c_ref, FP64 [n] (network input channel)
    // per-axis stencil coefficients: y = E u[i+1] + W u[i-1] + N u[j+1] + S u[j-1] + (k^2 - dx - dy) u
    // forward (A) and adjoint (A^H) sets, in FP64 and FP32
    double2 *fE_d, *fW_d, *fN_d, *fS_d, *aE_d, *aW_d, *aN_d, *aS_d, *dx_d, *dy_d;
    float2 *fE_f, *fW_f, *fN_f, *fS_f, *aE_f, *aW_f, *aN_f, *aS_f, *dx_f, *dy_f;
    double *sigx, *sigy;  // PML damping at the nodes, [nxt], [nyt] (network input channels)
    // HZ_DISC_SPECTRAL: per-axis derivative tables d [nxt], [nyt] and M = G D G D [nxt][nxt],
    // [nyt][nyt] in FP64 and FP32 (NULL for finite differences)
    double *dtx, *dty;
    double2 *Mx_d, *My_d;
    float2 *Mx_f, *My_f;
    void* block;          // the single device allocation holding all of the above
    uint64_t uid = 0;     // handle identity (next_handle_uid)
};

namespace hz {

struct StencilCoef {
    const void *E, *W, *N, *S, *dx, *dy;
    const void* k2;
    int conj_diag;
};
StencilCoef stencil_coef(const hz_problem* p, bool fp64, bool adjoint);
// true when the FP32 operator can run two points per lane on x -> y (even row length, 16-byte
// aligned vectors)
bool stencil_pairs_ok(const hz_problem* p, const void* x, const void* y);

// y = A x (or A^H x) in the precision of the complex type (float2 or double2).
int launch_stencil(const hz_problem* p, bool fp64, bool adjoint, const void* x, void* y, hipStream_t s,
                   const int* skip = nullptr);
// r = b - A x in FP64 (b, x, r: double2 [n]); writes one ||r||^2 partial per block to part
// (block count = stencil_blocks(p)).
int launch_resid64(const hz_problem* p, const double2* b, const double2* x, double2* r,
                   double* part, const int* skip, hipStream_t s);
int stencil_blocks(const hz_problem* p);
inline bool is_spectral(const hz_problem* p) { return p->g.disc == HZ_DISC_SPECTRAL; }
// Fourier-differentiation operator (spectral.hip): setup at creation, y = A x / A^H x, and the FP64
// residual r = b - A x with one ||r||^2 partial per tile (spectral_blocks of them)
int spectral_setup(hz_problem* p, hipStream_t s);
int spectral_blocks(const hz_problem* p);
int launch_spectral(const hz_problem* p, bool fp64, bool adjoint, const void* x, void* y, hipStream_t s,
                    const int* skip = nullptr);
// FP32 form of the residual with partials (the training loss on the spectral operator)
int launch_spectral_resid32(const hz_problem* p, const float2* b, const float2* x, float2* r, double* part,
                            const int* skip, hipStream_t s);
int launch_spectral_resid64(const hz_problem* p, const double2* b, const double2* x, double2* r, double* part,
                            const int* skip, hipStream_t s);
// y = b - A x in FP32 (float2 [n]) with one ||y||^2 partial (FP64) per block.
int launch_resid32(const hz_problem* p, const float2* b, const float2* x, float2* y, double* part, hipStream_t s);

}  // namespace hz
