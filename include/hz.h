/*
 * hz.h -- C ABI of the MI355X (gfx950) library for neural-operator-preconditioned
 * flexible GMRES on the 2-D heterogeneous Helmholtz equation with a PML.
 *
 * Method (paper: "Neural operator preconditioning from mixed dataset for the
 * Helmholtz equations", Sections 2-3): A(c) u = b with A = Laplacian + k^2,
 * k = omega / c (eq. (1), eq. (3)), a quadratic PML damping profile (eq. (2)),
 * solved by flexible GMRES (Algorithm 1, eq. (4)) whose preconditioner is a
 * U-Net neural operator z = N(v, c, sigma) (eq. (7), eq. (9)) trained with the
 * relative-residual loss (eq. (12)); stopping rule eq. (13).
 *
 * Conventions shared by every entry point
 *   - Grid: nx_t = nx + 2 npml nodes along x, ny_t = ny + 2 npml along y,
 *     n = nx_t * ny_t. Grid vectors are row-major with x fastest: entry
 *     (j, i) is at index j * nx_t + i.
 *   - Complex vectors are interleaved (re, im): HZ_C64 = two floats per entry
 *     (torch.complex64), HZ_C128 = two doubles (torch.complex128).
 *   - Every pointer named *_dev is device memory on the current HIP device.
 *     Host pointers are named *_host. The caller allocates and frees every
 *     input, output and workspace buffer; the library never frees caller
 *     memory. Handles own their own (immutable after creation) device data;
 *     a network handle also records the launch variants no_autotune chose (under a lock).
 *   - `stream` is a hipStream_t (NULL = the default stream). All calls are
 *     asynchronous on `stream` except fgmres_solve / fgmres_solve_batched,
 *     which synchronise `stream` once per restart cycle and return after
 *     completion, and the *_create calls, which synchronise once.
 *   - Return value: HZ_OK (0), HZ_NOT_CONVERGED (1, not an error: the info
 *     record is filled) or a negative error code. Arguments are validated
 *     before any launch; on error nothing is launched and hz_last_error()
 *     (thread-local) describes the failure. No C++ exception crosses the ABI.
 *   - Apart from those launch choices handles are read-only after creation:
 *     concurrent calls on different streams with different workspaces are safe
 *     (no_set_layer_variant and no_set_fused_upsampling excepted, see there).
 */
#ifndef HZ_H
#define HZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HZ_OK               0
#define HZ_NOT_CONVERGED    1
#define HZ_ERR_ARG         -1   /* invalid argument (NULL pointer, bad size, unsupported combination) */
#define HZ_ERR_HIP         -2   /* a HIP runtime call failed */
#define HZ_ERR_WORKSPACE   -3   /* workspace smaller than the matching *_workspace_size */
#define HZ_ERR_BREAKDOWN   -4   /* FGMRES: Z_k lost rank (e.g. zero preconditioner output) */
#define HZ_ERR_NONFINITE   -5   /* NaN or Inf in the input or an iterate */

/* Complex element type of a vector argument. */
typedef enum { HZ_C64 = 0, HZ_C128 = 1 } hz_dtype;

/* Arithmetic of the neural operator: BF16 operands with FP32 accumulation on
 * MFMA, FP32 on MFMA, or FP64 on MFMA. */
typedef enum { NO_BF16 = 0, NO_FP32 = 1, NO_FP64 = 2 } no_prec;

/* ------------------------------------------------------------------ problem */

/* One discrete Helmholtz system (Section 2.1). Node spacing h, angular
 * frequency omega, PML of npml cells per side whose damping grows as
 * sigma_max * (depth / npml)^2 (eq. (2)) and stretches the derivatives by
 * 1 / (1 + i sigma / omega). Velocities are divided by c_ref (m/s) before use,
 * so k^2 = (omega * c_ref / c)^2. */
typedef struct {
    int32_t nx, ny;       /* interior cells along x and y (>= 1) */
    int32_t npml;         /* PML cells on each side (>= 0) */
    double h;             /* grid step (> 0) */
    double omega;         /* angular frequency (> 0); the paper uses 1 */
    double sigma_max;     /* damping at the outermost node (>= 0) */
    double c_ref;         /* reference speed in m/s (> 0) */
    int32_t disc;         /* HZ_DISC_FD (0, five-point finite differences, zero outside the grid)
                             or HZ_DISC_SPECTRAL (1, Fourier differentiation over the periodic
                             grid, the paper's discretization) */
} hz_grid;

#define HZ_DISC_FD       0
#define HZ_DISC_SPECTRAL 1

typedef struct hz_problem hz_problem;

/* Build the operator data of one system from the velocity field
 * c_dev (float32, [ny_t][nx_t], m/s, every entry > 0): k^2 in FP32 and FP64, the
 * per-axis PML coefficients at nodes and half-nodes, and the network's static
 * channels. Runs the setup kernels on `stream` and synchronises it.
 * Errors: HZ_ERR_ARG for a bad grid or NULL pointer, HZ_ERR_NONFINITE if some
 * c is not finite or not positive, HZ_ERR_HIP on allocation failure. */
int hz_problem_create(const hz_grid* grid, const float* c_dev, void* stream, hz_problem** out);
int hz_problem_destroy(hz_problem* p);
/* Number of grid nodes n = nx_t * ny_t and the totals nx_t, ny_t (any may be NULL). */
int hz_problem_dims(const hz_problem* p, int64_t* n, int32_t* nx_t, int32_t* ny_t);

/* y = A x (adjoint = 0) or y = A^H x (adjoint = 1), eq. (3). HZ_DISC_FD: the five-point
 * stretched Laplacian plus k^2 with zero values outside the grid. HZ_DISC_SPECTRAL (Section
 * 2.1, Table 1): A u = (1/gx) Dx((1/gx) Dx u) + (1/gy) Dy((1/gy) Dy u) + k^2 u with the periodic
 * spectral derivatives D (Nyquist mode zeroed for an even axis) and gamma = 1 + i sigma / omega
 * at the nodes; its setup forms the per-axis matrices (1/g) D (1/g) D once (O(N^3) work and
 * N^2 complex entries per axis, FP64 and FP32, at problem creation).
 * x_dev, y_dev: n complex entries of type `dtype` (must not overlap). */
int hz_op_apply(const hz_problem* p, hz_dtype dtype, int adjoint,
                const void* x_dev, void* y_dev, void* stream);

/* --------------------------------------------------------- neural operator */

/* Two U-Net layer sets (Section 3.1), chosen by `kind`:
 * NO_ARCH_UNET3 (0): `levels` resolution levels (levels - 1 average poolings),
 *   base channels doubling per level, 3x3 convolutions with ReLU, 2x2 stride-2
 *   transposed convolutions on the way up, skip connections by concatenation.
 * NO_ARCH_PAPER8 (1): Table 2's layers: `levels` = depth 8x8 stride-2 padding-3
 *   convolutions down and as many transposed ones up, `base` channels in every
 *   layer, PReLU (one slope per layer), batch normalisation folded into the
 *   convolutions; the decoder concatenates the encoder output of its input size
 *   (encoder part first). Inference only: no_loss_backward, the batched solver
 *   and the launch-variant calls reject it.
 * Both end in a 1x1 head with 2 outputs (Re, Im). in_ch = 2 takes the (scaled)
 * Re/Im of the field; in_ch = 5 adds c / c_ref, sigma_x, sigma_y. */
#define NO_ARCH_UNET3  0
#define NO_ARCH_PAPER8 1
typedef struct {
    int32_t levels;   /* UNET3: 1..6; PAPER8: depth 1..5 */
    int32_t base;     /* UNET3: base channels, a multiple of 8; PAPER8: 32 */
    int32_t in_ch;    /* 2 or 5 */
    int32_t kind;     /* NO_ARCH_UNET3 (0, also what a zero-initialised struct gives) or NO_ARCH_PAPER8 */
} no_arch;

typedef struct no_net no_net;

/* Number of float32 parameters of the flat parameter vector: per layer, in the
 * order enc0a, enc0b, enc1a, ..., then up(L-2), dec(L-2)a, dec(L-2)b, ..., up0,
 * dec0a, dec0b, head, the weight ([out][in][3][3] for 3x3 convolutions,
 * [in][out][2][2] for transposed convolutions, [out][in][1][1] for the head)
 * followed by its bias. PAPER8: down1..down(L), up(L-1), up(L-2), ..., up0, head,
 * each as its weight ([out][in][8][8] down, [in][out][8][8] up, [out][in][1][1]
 * head), its bias and (down, up) its PReLU slope; -1 for an unsupported arch. */
int64_t no_param_count(const no_arch* arch);

/* Create a network and load theta_dev (float32, no_param_count entries); the
 * library keeps its own repacked BF16, FP32 and FP64 copies. Synchronises. */
int no_net_create(const no_arch* arch, const float* theta_dev, void* stream, no_net** out);
/* Replace the parameters (asynchronous on `stream`). */
int no_net_set_weights(no_net* net, const float* theta_dev, void* stream);
int no_net_destroy(no_net* net);

/* Workspace bytes for no_precond_apply on this problem at this precision. */
size_t no_workspace_size(const no_net* net, const hz_problem* p, no_prec prec);

/* z = N(v, c, sigma), eq. (7): s = ||v|| / sqrt(n); the network runs on the
 * zero-padded channels [Re v / s, Im v / s (, c / c_ref, sigma_x, sigma_y)] and
 * z = s (out_0 + i out_1) on the grid (z = 0 when v = 0).
 * v_dev, z_dev: n complex entries of type `dtype`. ws_dev: ws_bytes bytes. */
int no_precond_apply(const no_net* net, const hz_problem* p, no_prec prec, hz_dtype dtype,
                     const void* v_dev, void* z_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same z = N(v, c, sigma) as no_precond_apply, with
 * the same kernels and result bits, but its scratch is a fixed library-owned array of
 * NO_NOALLOC_SCRATCH_BYTES bytes per GPU (held until the process ends) instead of a caller
 * workspace. Nothing is allocated: no hipMalloc / hipFree and no allocating library routine. The
 * caller still passes v_dev and z_dev (n complex entries of type `dtype`).
 * Every call on one GPU shares that GPU's array and leaves its contents behind, so calls that
 * overlap on one GPU (different host threads, or different streams without ordering) race;
 * serialise them. Nothing in the array needs to start at zero.
 * Errors: HZ_ERR_ARG (NULL pointer, bad dtype or precision, v == z), HZ_ERR_WORKSPACE when the grid
 * and precision need more scratch than the fixed size (no_workspace_size says how much; the
 * 4-level / 32-channel network needs about 45 MB in BF16 and 90 MB in FP32 at 296^2 nodes, so
 * BF16 fits up to about 500^2 nodes), HZ_ERR_HIP
 * when the array's device address cannot be found; nothing is launched on error. */
#define NO_NOALLOC_SCRATCH_BYTES (128ull << 20)
int no_precond_apply_noalloc(const no_net* net, const hz_problem* p, no_prec prec, hz_dtype dtype,
                             const void* v_dev, void* z_dev, void* stream);

/* Time every launch variant (output-channel tile, pixel-tile height, input-channel chunks per
 * LDS stage) of every 3x3 layer at this problem's padded size and precision, on the forward
 * workspace ws_dev
 * (no_workspace_size bytes), and keep the fastest in the network handle; later forward passes
 * at that size use it. The variants accumulate every output in the same order, so the choice
 * never changes a result bit. fgmres_solve calls it on its first use of a size.
 * Synchronises `stream`; returns at once if the size was tuned before. Thread-safe. */
int no_autotune(const no_net* net, const hz_problem* p, no_prec prec, void* ws_dev, size_t ws_bytes,
                void* stream);

/* Launch variant used for 3x3 layer `layer` at (batch, H, W, prec): output-channel tile *tn
 * (16, 32 or 64; 0 = the built-in choice), pixel-tile height *rows (8 or 16), input-channel
 * chunks per LDS stage *stages (1, 2 or 4: one global-load latency per stage) and pixel tiles per
 * workgroup *tiles (1; or 2 and more for the weight-stationary form, which keeps the weights of
 * its output channels in LDS across that many tiles; there *stages counts the tiles whose
 * patch loads are in flight together, 2 to 4), as no_autotune chose it or no_set_layer_variant
 * pinned it. Errors: NULL pointer, not a 3x3 layer. */
int no_layer_variant(const no_net* net, int layer, no_prec prec, int batch, int H, int W, int32_t* tn,
                     int32_t* rows, int32_t* stages, int32_t* tiles);

/* Pin the launch variant of 3x3 layer `layer` at (batch, H, W, prec) to (tn, rows, stages,
 * tiles), as if no_autotune had chosen it (a later no_autotune of that size keeps it). Every
 * variant gives the same result bits; this fixes the launch for profiling and measurement.
 * Errors: not a 3x3 layer, tn not in {16, 32, 64} or not dividing the stored output channels,
 * rows not 8 or 16, stages not 1, or 2 / 4 for BF16 where that many chunk buffers fit in the
 * 160 KB of LDS of a workgroup (4 with tn 16, or tn 32 and 8 rows), tiles not 1, or 2..64 for
 * BF16 where the layer's input is at most 4 whole chunks of 32 channels per part and the weights
 * and patches of all chunks fit in the LDS (then stages 2 or 3, or 4 with at most 2 chunks; 2
 * with 16 rows).
 * Thread-safe. */
int no_set_layer_variant(const no_net* net, int layer, no_prec prec, int batch, int H, int W, int tn, int rows,
                         int stages, int tiles);

/* Choose how no_precond_apply and fgmres_solve run a decoder level with BF16 activations
 * whose coarser tensor has at most 128 channels: the fused form computes the 2x2 stride-2
 * transposed convolution (the decoder's upsampling, Section 3.1) inside the blocks of the
 * level's first 3x3 convolution instead of storing it. mode 0: never; 1: always where it
 * applies; 2 (the default): where no_autotune measured it faster than the two separate layers
 * (untuned sizes run them separately). Every choice gives the same result bits. Not
 * thread-safe against concurrent solves on the handle. Errors: NULL network, mode not 0-2. */
int no_set_fused_upsampling(no_net* net, int mode);

/* Shape of layer `layer` (0-based, in the order of the flat parameter vector):
 * kind 0 = 3x3 convolution + ReLU, 1 = 2x2 stride-2 transposed convolution, 2 = 1x1 head,
 * 3 = 8x8 stride-2 convolution + PReLU, 4 = 8x8 stride-2 transposed convolution + PReLU;
 * cin_p / cout_p = input / output channels as stored (zero-padded to a multiple of 16, the
 * network input to 8); cat_cp = stored channels of the first part of a concatenated input
 * (0 if the input is not a concatenation). Any output pointer may be NULL. */
int no_layer_info(const no_net* net, int layer, int32_t* kind, int32_t* cin_p, int32_t* cout_p,
                  int32_t* cat_cp);

/* Run one 3x3, transposed-convolution or 8x8 layer of the network on caller activations, as the
 * forward pass does (with the launch variant no_autotune chose for this layer and size, if any).
 * x0_dev: [batch][H][W][c0] with c0 = cat_cp for a concatenated input and c0 = cin_p otherwise;
 * x1_dev: [batch][H][W][cin_p - cat_cp] (second part) or NULL; y_dev: [batch][H'][W'][cout_p]
 * with (H', W') = (H, W) for a 3x3 layer, (2H, 2W) for a transposed one (2x2 or 8x8) and
 * (H/2, W/2) for an 8x8 stride-2 convolution (H, W even); pool_dev: optional
 * [batch][H/2][W/2][cout_p] average-pooled copy of y (3x3 layers, H and W even). Elements are
 * BF16 (raw 16-bit), float or double per `prec`. ws_dev / ws_bytes: scratch for a split of the
 * input channels (4 x batch x H x W x cout_p accumulators; NULL disables the split).
 * Meant for per-layer tests and profiling. */
int no_layer_forward(const no_net* net, int layer, no_prec prec, int batch, int H, int W,
                     const void* x0_dev, const void* x1_dev, void* y_dev, void* pool_dev,
                     void* ws_dev, size_t ws_bytes, void* stream);

/* Workspace bytes for no_loss_backward with `batch` samples on problems of one size and the
 * same `recompute` setting. */
size_t no_train_workspace_size(const no_net* net, const hz_problem* p, int batch, no_prec prec,
                               int recompute);

/* Physics-informed loss and its gradient (eq. (10)-(12)) for a batch of residuals:
 * per sample q_b = A_b N(r_b) - r_b and l_b = ||q_b|| / ||r_b|| (squared != 0:
 * ||q_b||^2 / ||r_b||^2); loss = mean_b l_b. Reverse mode through A^H and the
 * U-Net. problems: `batch` handles of one grid size and one discretization (the five-point
 * stencil, or the Fourier-differentiation operator of Section 2.1 with its adjoint); r_dev:
 * [batch][n] complex64;
 * loss_dev: 1 float (written); per_sample_dev: `batch` floats or NULL;
 * grad_dev: no_param_count floats (overwritten with d loss / d theta), or NULL to evaluate the
 * loss alone (a validation pass: the forward pass and the residuals, no reverse pass).
 * prec: NO_BF16 (BF16 operands, FP32 accumulation) or NO_FP32. recompute != 0 checkpoints
 * activations for large grids: the forward pass keeps only each level's outputs (and pooled
 * inputs), and the first-convolution and upsampled tensors of a level are recomputed with the
 * same kernels just before that level's backward step, so loss and gradient are bit-identical
 * to recompute = 0 with a smaller workspace. Asynchronous on `stream`, except that the first
 * call at a (grid size, batch) autotunes the forward layers as no_autotune does (which
 * synchronises the stream once). */
int no_loss_backward(const no_net* net, int batch, const hz_problem* const* problems,
                     const void* r_dev, int squared, int recompute, no_prec prec,
                     float* loss_dev, float* per_sample_dev, float* grad_dev,
                     void* ws_dev, size_t ws_bytes, void* stream);

/* One Adam step on the float32 master parameters (Section 3.4), with the gradient
 * clipped to global L2 norm `clip` when clip > 0; refreshes the network's
 * working copies. theta/m/v/grad: no_param_count floats on the device; step >= 1. */
int no_adam_step(no_net* net, float* theta_dev, float* m_dev, float* v_dev, const float* grad_dev,
                 int step, float lr, float beta1, float beta2, float eps, float clip,
                 void* ws_dev, size_t ws_bytes, void* stream);
size_t no_adam_workspace_size(const no_net* net);

/* ------------------------------------------------------------------- solver */

typedef struct {
    int32_t m;            /* cycle length (restart), >= 1 */
    int32_t maxit;        /* cap on preconditioner applications, >= 1 */
    double tol;           /* relative residual target (eq. (13)), > 0 */
    hz_dtype krylov;      /* HZ_C64: FP32 Krylov basis; HZ_C128: FP64 */
    no_prec net_prec;     /* arithmetic of the network (ignored when net is NULL) */
    double* hist_host;    /* optional: |g_{j+1}| / ||b|| after every iteration */
    int32_t hist_len;     /* entries available in hist_host */
    int32_t ortho;        /* 0: CGS with one reorthogonalisation (three reductions per step);
                             1: delayed reorthogonalisation (one reduction per step: the step's
                             reduction also reorthogonalises and normalises the previous vector,
                             whose network input scale is its exact norm, summed from partials
                             that the step's update pass leaves behind); needs a network and
                             fgmres_solve; same iterates in exact arithmetic */
} hz_opts;

/* Phases of a solve timed into hz_info.phase_ms (milliseconds; Section 4 reports the
 * elapsed time of a solve, ET): */
enum {
    HZ_PHASE_SETUP = 0,   /* GPU time from the start of the solve to the first basis vector: the
                             network's launch-variant trials on the first call at a grid size,
                             ||b||, the FP64 residual b - A x0 and v_1 */
    HZ_PHASE_CYCLES = 1,  /* GPU time of the restart cycles (network, matvec, Gram-Schmidt and
                             Hessenberg steps, cycle end with the FP64 true residual) */
    HZ_PHASE_BUILD = 2,   /* host time spent capturing and instantiating cycle graphs (zero when
                             every cycle replays a kept graph) */
    HZ_PHASE_TOTAL = 3,   /* host wall time of the whole call */
    HZ_NPHASE = 4
};

typedef struct {
    int32_t status;       /* HZ_OK, HZ_NOT_CONVERGED, HZ_ERR_BREAKDOWN or HZ_ERR_NONFINITE */
    int32_t its;          /* preconditioner applications (Arnoldi steps) */
    int32_t cycles;       /* restart cycles started */
    double est_relres;    /* last Givens estimate |g_{j+1}| / ||b|| */
    double true_relres;   /* FP64 ||b - A x|| / ||b|| of the returned x */
    double phase_ms[HZ_NPHASE];   /* phase times (HZ_PHASE_*); the batched solve writes the
                                     batch's times into every record */
} hz_info;

/* Workspace bytes for fgmres_solve. */
size_t fgmres_workspace_size(const hz_problem* p, const no_net* net, const hz_opts* opts);

/* Solve A x = b by restarted flexible GMRES(m), Algorithm 1, right-preconditioned
 * by the network (net == NULL: identity, i.e. plain GMRES). Each cycle starts
 * from the FP64 true residual r = b - A x, builds V and Z with Gram-Schmidt
 * orthogonalisation (CGS with one reorthogonalisation), keeps the Hessenberg
 * least-squares problem in FP64 with complex Givens rotations, ends early when
 * |g_{j+1}| / ||b|| <= tol, and adds Z y to x in FP64. Converged means the FP64
 * true residual <= tol. b_dev: n complex128 (read); x_dev: n complex128, read as
 * x0 and overwritten with the solution. info_host: filled on return.
 * Returns HZ_OK, HZ_NOT_CONVERGED or an error (the info record says which). */
int fgmres_solve(const hz_problem* p, const no_net* net, const hz_opts* opts,
                 const void* b_dev, void* x_dev, void* ws_dev, size_t ws_bytes,
                 hz_info* info_host, void* stream);

/* Batched solve of nsys independent systems of (possibly) different grid sizes
 * that share one network and one set of options: the systems advance together,
 * one network launch and one set of Krylov launches per step covering every
 * active system; systems leave the batch as they converge. b_dev[s], x_dev[s]:
 * complex128 vectors of system s. info_host: nsys records. */
size_t fgmres_batched_workspace_size(int nsys, const hz_problem* const* problems,
                                     const no_net* net, const hz_opts* opts);
int fgmres_solve_batched(int nsys, const hz_problem* const* problems, const no_net* net,
                         const hz_opts* opts, const void* const* b_dev, void* const* x_dev,
                         void* ws_dev, size_t ws_bytes, hz_info* info_host, void* stream);

/* Description of the last error on this thread ("" if none). */
const char* hz_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HZ_H */
