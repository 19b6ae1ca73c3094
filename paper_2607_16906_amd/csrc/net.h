// Internal view of the neural-operator handle and its forward/backward entry points.
#pragma once

#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"
#include "net_kernels.h"
#include "problem.h"

namespace hz {

// L_DOWN8 / L_UP8: the 8x8 stride-2 layers of the paper's own network (NO_ARCH_PAPER8)
enum LayerKind { L_CONV3 = 0, L_CONVT2 = 1, L_CONV1 = 2, L_DOWN8 = 3, L_UP8 = 4 };

struct Layer {
    int kind;
    int cin, cout;          // logical channels
    int cin_p, cout_p;      // channels as stored (padded to a multiple of 8 / 16)
    int cat_c, cat_cp;      // concatenated input: logical / stored channels of the first part (0: none)
    int64_t w_off, b_off;   // offsets in the flat FP32 parameter vector
    int64_t pk_off;         // offset of the repacked weights (elements) in the packed buffers
    int64_t pk_len;         // repacked weight elements
    int64_t bias_off;       // offset of the bias in the packed bias buffers
    int64_t a_off = -1;     // PReLU slope in the flat vector (L_DOWN8 / L_UP8; stored at bias[cout_p])
};

// 8x8 stride-2 padding-3 convolution (up = false: y is [Hin/2][Win/2]) or transposed convolution
// (up = true: y is [2 Hin][2 Win]) of concat[x0, x1] (x1 = NULL and cat_cp = 0 without a second
// part), + bias, then PReLU with slope bias[cout_p]; w packed [64 taps][wcout][cin_p] (the 32
// output channels are the first rows of each tap; wcout >= 32); 32 output channels; ypre (optional)
// receives the pre-activation values (defined in net8.hip).
template <class P>
int launch_conv8(bool up, const typename P::T* x0, const typename P::T* x1, int cin_p, int cat_cp,
                 const typename P::T* w, const typename P::Acc* bias, typename P::T* y, int cout_p, int Hin, int Win,
                 int batch, const int* skip, hipStream_t s, typename P::T* ypre = nullptr, int wcout = 32);

}  // namespace hz

struct no_net {
    no_arch a;
    int64_t nparam;
    std::vector<hz::Layer> layers;   // order of the flat parameter vector
    int64_t pk_total;                // repacked weight elements
    int64_t bias_total;              // packed bias elements
    hz::bf16_t* w_bf;                // repacked weights, BF16
    float* w_f32;                    // repacked weights, FP32
    double* w_f64;                   // repacked weights, FP64
    hz::bf16_t* wt_bf;               // data-gradient packs (flipped / transposed), BF16
    float* wt_f32;
    double* wt_f64;
    float* b_f32;                    // biases (FP32; the BF16 path adds them in FP32)
    double* b_f64;
    void* block;
    hz::Layer* layers_dev;           // device copy of `layers` (for the one-launch repack)
    int64_t* repack_start;           // device: first repack block of each layer, then the total
    int64_t repack_blocks;           // repack blocks over all layers
    // autotuned launch variants of the 3x3 layers, keyed by (layer, H, W, batch, precision)
    std::map<std::array<int, 5>, hz::ConvCfg> tuned;
    std::mutex tune_mu;
    int fuse_up = 2;   // fused decoder convolution: 0 never, 1 where it applies, 2 where autotuned faster
    uint64_t uid = 0;  // handle identity (next_handle_uid)
    // launch-choice generation: advanced whenever a variant is pinned, a size is newly tuned or the
    // fused-upsampling mode changes, so that kept solver graphs recorded with older choices are
    // not replayed
    std::atomic<uint64_t> tune_gen{0};
};

namespace hz {

int net_level_count(const no_net* net);
// Padded grid of the network for a problem (multiple of 2^(levels-1)).
void net_padded_dims(const no_net* net, const hz_problem* p, int* Hp, int* Wp);
size_t net_fwd_ws_bytes(const no_net* net, int Hp, int Wp, int batch, no_prec prec);
// z = N(v) for one field (c128: complex128 vectors, else complex64). skip: optional device flag.
// unit_norm: v is a Krylov vector of norm 1, so s = 1 / sqrt(n) without a reduction.
// vscale (device scalar, with unit_norm only): v is first scaled in place by *vscale, which
// makes it of norm 1 (the Arnoldi normalisation v_{j+1} = w / h_{j+1,j} done here).
// ||v||^2 given as partial sums by the caller's last pass over v: part[q * ldp].x, q < count;
// sc (device, 2 doubles) receives [s, 1/s].
struct NormParts {
    const double2* part;
    int count, ldp;
    double* sc;
};
// nparts (without unit_norm and vscale): the input scale comes from the caller's partial sums
// and no separate reduction runs.
int net_precond(const no_net* net, const hz_problem* p, no_prec prec, bool c128, const void* v, void* z,
                void* ws, size_t ws_bytes, const int* skip, hipStream_t s, bool unit_norm = false,
                const double* vscale = nullptr, const NormParts* nparts = nullptr);
// Time every launch variant of every 3x3 layer at this problem's size (batch 1) on the forward
// workspace and remember the fastest; returns HZ_OK at once when already tuned. Synchronises.
int net_autotune(const no_net* net, const hz_problem* p, no_prec prec, void* ws, size_t ws_bytes, hipStream_t s);
hz::ConvCfg net_cfg(const no_net* net, int layer, int H, int W, int batch, no_prec prec);
// launch variant of the fused form (transposed convolution inside) of decoder 3x3 layer `layer`
hz::ConvCfg net_cfg_up(const no_net* net, int layer, int H, int W, int batch, no_prec prec);

}  // namespace hz
