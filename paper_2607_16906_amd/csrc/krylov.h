// Internal launchers of the Arnoldi / least-squares kernels used by the FGMRES driver.
#pragma once

#include "common.h"

namespace hz {

// Device-resident state of one solve; the host reads it once per restart cycle.
struct SolveState {
    double bnorm;      // ||b||
    double tol;
    double beta;       // ||r|| at the start of the current cycle
    double true_rel;   // ||b - A x|| / ||b|| of the current x
    double est;        // last Givens estimate |g_{j+1}| / ||b||
    double wnorm0;     // ||A z_j|| before orthogonalisation (breakdown test)
    double inv_h;      // 1 / h_{j+1,j} (scales v_{j+1})
    double inv_beta;   // 1 / beta (scales v_1)
    int m;
    int stop;          // nonzero: the remaining steps of this cycle are skipped
    int k;             // Arnoldi columns completed in this cycle
    int its;           // preconditioner applications so far
    int cycles;        // cycles started
    int flags;         // FL_* bits
    int hist_cap;
    int pad_;
};
enum { FL_BREAKDOWN = 1, FL_NONFINITE = 2, FL_CONVERGED = 4 };

// Per-solve buffers carved from the caller workspace.
struct KrylovBufs {
    SolveState* st;
    double2* R;        // (m+1) x m upper-triangularised Hessenberg, column-major
    double* cs;        // m
    double2* sn;       // m
    double2* g;        // m+1
    double2* y;        // m
    double2* h1;       // m+2 (slot m+1 holds a squared norm in .x)
    double2* h2;       // m+2
    double2* part;     // nblk x ldp partial sums
    int ldp;           // m + 2
    double* hist;      // hist_cap entries
    int hist_cap;
    // delayed reorthogonalisation (one reduction per step)
    double2* pend;     // m+1: first-pass entries of the column completed at the next step
    double2* colb;     // m+1: the column being completed
    double2* coef;     // 2m+2: coefficients of the update pass
    double* lag_sc;    // 4: network input scale s, 1/s; ||w|| of this and of the previous step
};

struct Split {
    int nblk;
    int64_t per_block;
};
Split krylov_split(int64_t n);

// ||x||^2 partials of a complex vector (float2 or double2) into part[b * ldp + slot].x
int launch_norm_partials(bool c128, const void* x, int64_t n, Split sp, double2* part, int ldp, int slot,
                         const int* skip, hipStream_t s);
// out[i] = sum_b part[b * ldp + i] for i < cnt, fixed order
int launch_finalize(const double2* part, int nblk, int ldp, int cnt, double2* out, const int* skip, hipStream_t s);
// part[b][i] = sum over block b of conj(V_i) w (i < nv), plus ||w||^2 in slot nv when with_norm
int launch_dots(bool c128, const void* V, int64_t ldv, int nv, const void* w, int64_t n, Split sp,
                double2* part, int ldp, bool with_norm, const int* skip, hipStream_t s);

// w = A z (the problem's operator) fused with launch_dots(..., with_norm = true) on w; two: the
// sums are taken against both V_{nv-1} and w (slots 0..nv-1 and nv..2nv-1, ||w||^2 in slot 2nv)
int launch_stencil_dots(const hz_problem* p, bool c128, const void* z, const void* V, int64_t ldv, int nv,
                        void* w, Split sp, double2* part, int ldp, const int* skip, hipStream_t s,
                        bool two = false);
// delayed reorthogonalisation: the Hessenberg step (one block) and the one-pass update of step j
int launch_arnoldi_lag(KrylovBufs& kb, int j, bool tail, hipStream_t s);
int launch_update_lag(bool c128, void* V, int64_t ldv, int j, const double2* coef, int64_t n, Split sp,
                      double2* part, int ldp, const int* skip, hipStream_t s);
// w -= sum_i V_i h_i; mode 1 then also writes dots conj(V_i) w (slots 0..nv-1);
// mode 2 writes ||w||^2 into slot 0
int launch_update(bool c128, const void* V, int64_t ldv, int nv, const double2* h, void* w, int64_t n,
                  Split sp, double2* part, int ldp, int mode, const int* skip, hipStream_t s);

int launch_init_state(KrylovBufs& kb, int nblk, double tol, int m, hipStream_t s);
int launch_arnoldi_finish(KrylovBufs& kb, int j, int nblk, bool reorth, hipStream_t s);
int launch_scale(bool c128, void* v, int64_t n, const double* inv, const int* skip, hipStream_t s);
int launch_cycle_start(KrylovBufs& kb, const double* resid_part, int nparts, hipStream_t s);
int launch_cast_scale(bool c128, const double2* r, void* v, int64_t n, const SolveState* st, hipStream_t s);
int launch_backsolve(KrylovBufs& kb, hipStream_t s);
int launch_xupdate(bool c128, const void* Z, int64_t ldz, double2* x, int64_t n, const KrylovBufs& kb,
                   hipStream_t s);

}  // namespace hz
