// MFMA policies and the U-Net layer kernels (forward), shared by inference and training.
//
// Activations are NHWC with channels padded to a multiple of 8; a batch of
// fields is stored sample after sample. A 3x3 convolution is an implicit GEMM
// with M = output channels, N = pixels and K = 9 x input channels: each block
// owns an 8 x 16 pixel tile and TN output channels, stages the (8+2) x (16+2)
// input patch and the matching weights chunk by chunk in LDS, and feeds the
// matrix cores with 16 x 16 output blocks (rows = output channels, columns =
// 16 consecutive pixels of one image row). The epilogue adds the bias, applies
// ReLU and can also write the 2 x 2 average pool of the result.
#pragma once

#include <type_traits>

#include "common.h"

namespace hz {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(4))) float f32x4_t;
typedef __attribute__((ext_vector_type(4))) double f64x4_t;

// Lane layout of the 16x16 MFMA forms used here (64 lanes, l = lane):
//   A (16 x K): lane l holds row l % 16, k-group l / 16 (GW consecutive k);
//   B (K x 16): lane l holds column l % 16, k-group l / 16;
//   D (16 x 16): lane l holds rows 4 (l / 16) + r, r = 0..3, of column l % 16
//   for the FP32-accumulating forms, and rows (l / 16) + 4 r for the FP64 form
//   (row_of gives the row of accumulator register r).
struct PolBF16 {
    using T = bf16_t;
    using Acc = float;
    using AccV = f32x4_t;
    using Frag = bf16x8_t;
    static constexpr int GW = 8;    // k per lane per MFMA
    static constexpr int CK = 32;   // channels per LDS chunk
    __device__ static Frag load(const T* p) { return __builtin_bit_cast(Frag, *(const uint4*)p); }
    __device__ static Frag zero() { return __builtin_bit_cast(Frag, uint4{0, 0, 0, 0}); }
    __device__ static AccV mma(Frag a, Frag b, AccV c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static T cvt(Acc v) { return f2bf(v); }
    __device__ static Acc val(T v) { return bf2f(v); }
    __device__ static int row_of(int lg, int r) { return 4 * lg + r; }
    // the 4 registers of a lane are 4 consecutive channels: one 8-byte store at p = &row_of(lg, 0)
    static constexpr bool CONTIG = true;
    __device__ static void store4(T* p, const Acc (&v)[4]) {
        uint2 u;
        u.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
        u.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
        *(uint2*)p = u;
    }
};

struct PolF32 {
    using T = float;
    using Acc = float;
    using AccV = f32x4_t;
    using Frag = float;
    static constexpr int GW = 1;
    static constexpr int CK = 16;
    __device__ static Frag load(const T* p) { return *p; }
    __device__ static Frag zero() { return 0.0f; }
    __device__ static AccV mma(Frag a, Frag b, AccV c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static T cvt(Acc v) { return v; }
    __device__ static Acc val(T v) { return v; }
    __device__ static int row_of(int lg, int r) { return 4 * lg + r; }
    static constexpr bool CONTIG = true;   // one 16-byte store
    __device__ static void store4(T* p, const Acc (&v)[4]) { *(float4*)p = float4{v[0], v[1], v[2], v[3]}; }
};

struct PolF64 {
    using T = double;
    using Acc = double;
    using AccV = f64x4_t;
    using Frag = double;
    static constexpr int GW = 1;
    static constexpr int CK = 8;
    __device__ static Frag load(const T* p) { return *p; }
    __device__ static Frag zero() { return 0.0; }
    __device__ static AccV mma(Frag a, Frag b, AccV c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static T cvt(Acc v) { return v; }
    __device__ static Acc val(T v) { return v; }
    __device__ static int row_of(int lg, int r) { return lg + 4 * r; }
    static constexpr bool CONTIG = false;  // channels lg, lg + 4, ...: element stores
    __device__ static void store4(T* p, const Acc (&v)[4]) {
        for (int r = 0; r < 4; ++r) p[4 * r] = v[r];
    }
};

// y[row_of(lg, r)] = cvt(v[r]) for r < 4, with y = p - row_of(lg, 0)
template <class P>
__device__ __forceinline__ void store_rows(typename P::T* p, const typename P::Acc (&v)[4]) { P::store4(p, v); }

// One block of a ragged batch: system index, output-channel block start, tile origin (3x3:
// pixel row / column of an 8 x 16 tile; transposed conv: input row / first column of 64).
struct TileJob {
    int sys, c0, ty0, tx0;
};
// Per-system tensors of one layer in a ragged batch.
struct LayerIO {
    const void* x0;
    const void* x1;
    void* y;
    void* ypool;
    int H, W;
    const int* stop;   // the system's stop flag (the block returns when it is set)
    // fused 1x1 head (last 3x3 layer only): column col of z, i.e. z + col * zld, of nyt x nxt
    // points, scaled by sc[0]; element type float2 or double2 as the launch says
    void* z;
    int64_t zld;
    int nxt, nyt;
    const double* sc;
};

// Optional extras of a 3x3 convolution launch: a split of the output channels into two
// tensors (channels [0, split) -> y, [split, cout) -> y1) and ReLU masks for either part
// (an output entry is zeroed where the mask entry is <= 0). Used by the data gradient.
struct Conv3Out {
    int split = 0;
    void* y1_ = nullptr;
    const void* mask0_ = nullptr;
    const void* mask1_ = nullptr;
    // 1x1 output head fused into the epilogue (one block then covers every output channel and
    // y is not stored): z[yy * head_nxt + xx] = s (head_b + head_w ReLU(y)) as a complex number
    // (real, imaginary = head outputs 0, 1) for yy < head_nyt, xx < head_nxt, with y rounded to
    // the activation type first; s = head_fixed_s if > 0, else head_sc[0].
    const void* head_w = nullptr;   // activation type, [2][cout_p]
    const void* head_b = nullptr;   // accumulator type, [2]
    void* head_z = nullptr;         // float2 (head_c128 = 0) or double2
    int head_c128 = 0;
    int head_nxt = 0, head_nyt = 0;
    const double* head_sc = nullptr;
    double head_fixed_s = 0.0;
};

// Variant of a 3x3 convolution launch: channel tile (16 / 32 / 64; 0 = heuristic), rows per
// wavefront (2 or 4: 8- or 16-row pixel tiles), the number of input-channel splits (split-K
// writes FP32/FP64 partial sums to a workspace and reduces them in a separate epilogue kernel)
// and, for a decoder's first layer, whether the fused form is faster.
struct ConvCfg {
    int tn = 0;
    int rpw = 2;
    int ksplit = 1;
    int fuse = 0;   // decoder layer: take the fused form (transposed convolution inside, UpIn)
    int ns = 1;     // input-channel chunks per LDS stage (1, 2 or 4; BF16 only, same result bits)
    int tpb = 0;    // > 1: weight-stationary form with tpb pixel tiles per block (BF16, conv3_ws_ok);
                    // ns is then the number of tiles whose loads are in flight (2, 3 or 4)
};

// LDS bytes of the weight-stationary 3x3 form: the weights of wch chunks and two patch buffers of
// wch chunks each.
template <class P>
constexpr int conv3_ws_lds(int tn, int rpw, int wch) {
    const int ps = P::CK + 16 / (int)sizeof(typename P::T);
    return wch * (2 * (4 * rpw + 2) * 18 * ps + 9 * tn * ps) * (int)sizeof(typename P::T);
}

// An input of one k-group (P::GW channels) per tap, as the first layer's: the weight-stationary
// form then stages one k-group per pixel and runs conv3_tile's grouped-tap steps.
template <class P>
constexpr bool conv3_ws_small(int c0, int c1) {
    return c1 == 0 && c0 == P::GW;
}

// Whether the weight-stationary form applies: BF16, channel tile tn in {16, 32, 64} dividing
// cout_p, both input parts whole chunks of P::CK channels (1, 2 or 4 chunks) or an input of one
// k-group per tap (conv3_ws_small), and the LDS of all chunk buffers within 160 KB.
template <class P>
constexpr bool conv3_ws_ok(int tn, int rpw, int c0, int c1, int cout_p) {
    if (!std::is_same<P, PolBF16>::value) return false;
    if (tn != 16 && tn != 32 && tn != 64) return false;
    if (cout_p % tn) return false;
    if (conv3_ws_small<P>(c0, c1)) return conv3_ws_lds<P>(tn, rpw, 1) <= 160 * 1024;
    if (c0 % P::CK || c1 % P::CK || c0 + c1 == 0) return false;
    const int nch = (c0 + c1) / P::CK;
    if (nch != 1 && nch != 2 && nch != 4) return false;
    return conv3_ws_lds<P>(tn, rpw, nch) <= 160 * 1024;
}

// Whether a 3x3 launch with channel tile tn, rows per wavefront rpw and ns chunks per LDS stage
// exists: ns = 1 always; ns = 2 for BF16; ns = 4 for BF16 where the four stages fit in the LDS
// (160 KB per workgroup).
template <class P>
constexpr bool conv3_stages_ok(int tn, int rpw, int ns) {
    if (ns == 1) return true;
    if (ns != 2 && ns != 4) return false;
    if (!std::is_same<P, PolBF16>::value) return false;
    const int ps = P::CK + 8;   // BF16 pixel stride (elements)
    const int bytes = ((4 * rpw + 2) * 18 * ps + 9 * tn * ps) * 2;
    return ns * bytes <= 160 * 1024;
}

// Second input part of a decoder 3x3 convolution given as the 2x2 stride-2 transposed
// convolution of a coarser tensor, computed inside each block and never stored:
// U[2i+a][2j+b][c] = bt[c] + sum_k d[i][j][k] wt[2a+b][c][k], d: [H/2][W/2][cd] per sample.
struct UpIn {
    const void* d = nullptr;
    int cd = 0;
    const void* wt = nullptr;   // activation type, [4][c1][cd] (the transposed layer's pack)
    const void* bt = nullptr;   // accumulator type, [c1]
};
constexpr int UP_CDMAX = 128;   // largest coarse channel count of the fused form

// Host-side launch helpers (defined in net_fwd.hip), one per precision.
// conv3: y = act(conv3x3(concat[x0, x1]) + b) (+ pooled copy); batch samples along grid z.
template <class P>
int launch_conv3(const typename P::T* x0, int c0, const typename P::T* x1, int c1, const typename P::T* w,
                 const typename P::Acc* bias, typename P::T* y, int cout_p, typename P::T* ypool, int H, int W,
                 int batch, bool relu, const int* skip, hipStream_t s, Conv3Out ex = Conv3Out(),
                 ConvCfg cfg = ConvCfg(), typename P::Acc* splitbuf = nullptr);
// Ragged-batch versions: one launch over a job table (3x3: tiles of 4 rpw rows x 16 columns, rpw 2,
// or 4 with tn 32 in BF16).
template <class P>
int launch_conv3_jobs(const TileJob* jobs, int njobs, const LayerIO* io, const typename P::T* w,
                      const typename P::Acc* bias, int c0, int c1, int cout_p, int tn, int rpw, bool pool,
                      hipStream_t s);
// The same with the 1x1 output head fused into the epilogue (cout_p 16, 32 or 64, one job per
// pixel tile): writes column col of each system's z (LayerIO head fields) instead of y.
template <class P>
int launch_conv3_jobs_head(const TileJob* jobs, int njobs, const LayerIO* io, const typename P::T* w,
                           const typename P::Acc* bias, int c0, int c1, int cout_p, const typename P::T* head_w,
                           const typename P::Acc* head_b, int col, bool c128, hipStream_t s);
// Weight-stationary form over a job table (BF16, inputs of one or two chunks or of one k-group per
// tap; WSJ_TN output channels and 4 WSJ_RPW pixel rows per tile; job = (sys, first output channel, first tile, end tile) with tiles row-major over the
// system's image); with head_w the fused 1x1 head as in launch_conv3_jobs_head (cout_p == WSJ_TN).
constexpr int WSJ_TN = 32, WSJ_RPW = 4;
template <class P>
constexpr bool ws_jobs_ok(int c0, int c1, int cout_p) {
    return conv3_ws_ok<P>(WSJ_TN, WSJ_RPW, c0, c1, cout_p) && c0 + c1 <= 2 * P::CK;
}
// The data gradient of training (split output, masks, no bias) in the weight-stationary form:
// BF16, an input of 1 or 2 chunks, WSJ_TN-channel blocks that both output parts divide, 16 x 16
// tiles; y0 / y1 / masks as Conv3Out's split and masks, samples along grid z.
template <class P>
constexpr bool conv3_ws_dgrad_ok(int c0, int cout_p, int split) {
    return conv3_ws_ok<P>(WSJ_TN, WSJ_RPW, c0, 0, cout_p) && c0 <= 2 * P::CK && split % WSJ_TN == 0 &&
           (cout_p - split) % WSJ_TN == 0;
}
template <class P>
int launch_conv3_ws_dgrad(const typename P::T* x0, int c0, const typename P::T* w, typename P::T* y0, int cout_p,
                          int H, int W, int batch, int split, typename P::T* y1, const typename P::T* mask0,
                          const typename P::T* mask1, hipStream_t s);
template <class P>
int launch_conv3_ws_jobs(const TileJob* jobs, int njobs, const LayerIO* io, const typename P::T* w,
                         const typename P::Acc* bias, int c0, int c1, int cout_p, bool pool,
                         const typename P::T* head_w, const typename P::Acc* head_b, int col, bool c128,
                         hipStream_t s);
template <class P>
int launch_convT2_jobs(const TileJob* jobs, int njobs, const LayerIO* io, const typename P::T* w,
                       const typename P::Acc* bias, int cin_p, int cout_p, int tn, hipStream_t s);
// Weight-stationary transposed convolution over a job table (BF16, every input channel in one
// stage): job = (sys, first output channel, first 64-pixel input row segment, end segment), the
// segments of a system row-major (ceil(W / 64) per input row); tn 16 or 32.
template <class P>
constexpr bool convT2_ws_ok(int cin_p, int cout_p, int tn) {
    return std::is_same<P, PolBF16>::value && (tn == 16 || tn == 32) && cout_p % tn == 0 &&
           cin_p % (4 * P::GW) == 0 && cin_p > 0 && cin_p <= 4 * P::CK;
}
template <class P>
int launch_convT2_ws_jobs(const TileJob* jobs, int njobs, const LayerIO* io, const typename P::T* w,
                          const typename P::Acc* bias, int cin_p, int cout_p, int tn, hipStream_t s);
// channel tile chosen for a ragged batch (so that the job table can be built on the host)
int conv3_batch_tn(int cout_p, int64_t tiles);
int convT2_batch_tn(int cout_p);
template <class P>
int conv_chunk(int cin_p, int c0, int c1);
// Fused decoder convolution y = ReLU(conv3x3(concat[x0, U]) + b) with U = convT2(up) (see UpIn):
// the same result bits as launch_convT2 followed by launch_conv3. BF16 only; conv3_up_ok tells
// whether a layer qualifies.
template <class P>
bool conv3_up_ok(int c0, int c1, int cd, int H, int W);
template <class P>
int launch_conv3_up(const typename P::T* x0, int c0, UpIn up, int c1, const typename P::T* w,
                    const typename P::Acc* bias, typename P::T* y, int cout_p, int H, int W, int batch,
                    const int* skip, hipStream_t s, ConvCfg cfg);
// convT2: y[2i+a][2j+b] = sum_c x[i][j][c] w[a][b][.][c] + b
template <class P>
int launch_convT2(const typename P::T* x, int cin_p, const typename P::T* w, const typename P::Acc* bias,
                  typename P::T* y, int cout_p, int H, int W, int batch, const int* skip, hipStream_t s);

}  // namespace hz
