// U-Net layer kernels on the matrix cores (forward): 3x3 convolution as implicit
// GEMM with fused bias / ReLU / 2x2 average pool, and the 2x2 stride-2 transposed
// convolution. Templated over the arithmetic policy (BF16, FP32, FP64).
#include <type_traits>

#include "net_kernels.h"

namespace hz {

constexpr int CT = 256;        // threads per block (4 wavefronts)
constexpr int TW = 16;          // pixel tile width of the 3x3 convolution (rows: 4 per-wave row count)

// Consecutive workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Renumber the physical block id so that the blocks one XCD runs form one contiguous range of
// the logical order (in which blocks that read the same input tile are neighbours).
__device__ __forceinline__ int xcd_linear(int p, int n) {
    const int q = n / 8, r = n % 8;
    const int k = p % 8, i = p / 8;
    return k * q + (k < r ? k : r) + i;
}

template <class P>
constexpr int pix_stride() { return P::CK + 16 / (int)sizeof(typename P::T); }   // +16 B against bank conflicts

// The matrix-core work of one full input-channel chunk (P::CK channels) staged in LDS: patch
// pst ((4 RPW + 2) x 18 pixels, pixel stride pix_stride) and weights wst (9 taps x TN rows, same
// stride), accumulated into acc[pixel row][channel block] of the wavefront's RPW rows. Step st
// covers tap st / SPT and k-groups 4 (st mod SPT) + lg of it; all offsets are compile-time after
// unrolling (the reads of the next steps can be issued while the matrix cores work). The
// wavefront's RPW + 2 patch rows at the 3 column offsets are read from LDS once and shared by the
// 3 row offsets dy of the window; the accumulation order is tap by tap, k-groups within a tap.
template <class P, int TN, int RPW>
__device__ __forceinline__ void conv3_chunk_mma(typename P::AccV (&acc)[RPW][TN / 16], const typename P::T* pst,
                                                const typename P::T* wst, int wv, int lr, int lg) {
    using T = typename P::T;
    using Frag = typename P::Frag;
    constexpr int PS = pix_stride<P>();
    constexpr int NCB = TN / 16;
    constexpr int SPT = P::CK / P::GW / 4;
    const T* pbase = pst + ((RPW * wv) * (TW + 2) + lr) * PS + lg * P::GW;
    const T* wbase = wst + lr * PS + lg * P::GW;
    Frag b[RPW + 2][3][SPT];
#pragma unroll
    for (int ir = 0; ir < RPW + 2; ++ir)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
            for (int sg = 0; sg < SPT; ++sg)
                b[ir][dx][sg] = P::load(pbase + (ir * (TW + 2) + dx) * PS + 4 * sg * P::GW);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
#pragma unroll
        for (int sg = 0; sg < SPT; ++sg) {
            Frag a[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) a[cb] = P::load(wbase + (tap * TN + cb * 16) * PS + 4 * sg * P::GW);
#pragma unroll
            for (int pb = 0; pb < RPW; ++pb)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) acc[pb][cb] = P::mma(a[cb], b[pb + dy][dx][sg], acc[pb][cb]);
        }
    }
}

// The MFMA steps of an input of one k-group (P::GW channels) per tap held in LDS as conv3_chunk_mma's
// layout: step s takes taps 4 s .. 4 s + 3 (lane group lg: tap 4 s + lg, zero past the ninth), the
// same steps and operands as conv3_tile with a chunk of P::GW channels.
template <class P, int TN, int RPW>
__device__ __forceinline__ void conv3_group_mma(typename P::AccV (&acc)[RPW][TN / 16], const typename P::T* pst,
                                                const typename P::T* wst, int wv, int lr, int lg) {
    using Frag = typename P::Frag;
    constexpr int PS = pix_stride<P>();
    constexpr int NCB = TN / 16;
#pragma unroll
    for (int sp = 0; sp < 3; ++sp) {
        const int tap = 4 * sp + lg;
        Frag a[NCB], b[RPW];
        if (tap < 9) {
            const int dy = tap / 3, dx = tap - 3 * (tap / 3);
#pragma unroll
            for (int pb = 0; pb < RPW; ++pb) b[pb] = P::load(pst + ((RPW * wv + pb + dy) * (TW + 2) + lr + dx) * PS);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) a[cb] = P::load(wst + (tap * TN + cb * 16 + lr) * PS);
        } else {
#pragma unroll
            for (int pb = 0; pb < RPW; ++pb) b[pb] = P::zero();
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) a[cb] = P::zero();
        }
#pragma unroll
        for (int pb = 0; pb < RPW; ++pb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[pb][cb] = P::mma(a[cb], b[pb], acc[pb][cb]);
    }
}

// One block's tile: output channels [co0, co0 + TN) of the (4 RPW) x 16 pixel tile at (ty0, tx0)
// of sample bz, over the input-channel chunks [kbeg, kend). Each wavefront owns RPW rows of the
// tile. NS chunks form one stage: their patches and weights sit in NS LDS buffers, and the next
// stage's NS chunks are loaded into registers while the matrix cores work on the current stage
// (register double buffering), so that one global-load latency is paid per NS chunks. The chunks
// of a stage are computed one after the other in the order of NS = 1, so every NS gives the same
// result bits. With splitp set, the raw accumulators are written to splitp[[bz][pixel][channel]]
// (no bias or activation) for a later split-K reduction.
//
// UPCD > 0 (fused upsampling, see UpIn): the channels from c0 on are U, computed per chunk from the
// coarse patch d[ty0/2 - 1 .. ty0/2 + 2 RPW][tx0/2 - 1 .. tx0/2 + 8] (staged once in LDS, all
// up.cd <= UPCD channels): wavefront a' computes parity a' = 2a + b of the chunk's channels for
// every coarse pixel of the patch, with the same MFMA steps (input channels in groups of 4 GW, in
// order) as the stand-alone transposed convolution, adds the bias, rounds to the activation type
// and writes the values that land in the (4 RPW + 2) x 18 patch (zero outside the image).
template <class P, int TN, bool POOL, int RPW, int UPCD = 0, int NS = 1>
__device__ __forceinline__ void conv3_tile(const typename P::T* __restrict__ x0, int c0,
                                           const typename P::T* __restrict__ x1, int c1,
                                           const typename P::T* __restrict__ w,
                                           const typename P::Acc* __restrict__ bias,
                                           typename P::T* __restrict__ y, int cout_p,
                                           typename P::T* __restrict__ ypool, int H, int W, int relu, int ck,
                                           const Conv3Out& ex, int bz, int co0, int ty0, int tx0, int kbeg, int kend,
                                           typename P::Acc* __restrict__ splitp, UpIn up = UpIn(),
                                           const int* __restrict__ skip = nullptr) {
    using T = typename P::T;
    // the step-skip flag is read here but tested only once the first chunk's loads are in flight,
    // so that its memory latency overlaps theirs (nothing is written before the test)
    const int skipped = skip ? *skip : 0;
    using Acc = typename P::Acc;
    using AccV = typename P::AccV;
    using Frag = typename P::Frag;
    constexpr int TH_ = 4 * RPW;
    constexpr int PS = pix_stride<P>();
    constexpr int VE = 16 / sizeof(T);        // elements per 16-byte vector
    constexpr int NCB = TN / 16;              // output-channel blocks per block
    constexpr int VPP_MAX = P::CK / VE;
    constexpr int NPA = ((TH_ + 2) * (TW + 2) * VPP_MAX + CT - 1) / CT;   // patch vectors per thread
    constexpr int NPW = (9 * TN * VPP_MAX + CT - 1) / CT;                 // weight vectors per thread
    static_assert(NS == 1 || UPCD == 0, "multi-chunk stages are for the plain convolution");
    constexpr int PSZ = (TH_ + 2) * (TW + 2) * PS, WSZ = 9 * TN * PS;   // one chunk's patch / weights
    __shared__ __attribute__((aligned(16))) T patch[NS * PSZ];
    __shared__ __attribute__((aligned(16))) T wl[NS * WSZ];
    // fused upsampling: coarse patch geometry, LDS and per-lane fragments
    constexpr int DR = TH_ / 2 + 2, DC = TW / 2 + 2, NDP = DR * DC;   // coarse patch pixels
    constexpr int NDB = (NDP + 15) / 16;                               // their 16-pixel MFMA blocks
    constexpr int PSD = (UPCD > 0 ? UPCD : 0) + VE;                    // coarse pixel stride
    constexpr int NDV = UPCD > 0 ? (NDP * (UPCD / VE) + CT - 1) / CT : 1;
    constexpr int UMB = P::CK >= 16 ? P::CK / 16 : 1;                  // 16-channel blocks per chunk
    constexpr int UKS = UPCD > 0 ? UPCD / (4 * P::GW) : 1;             // MFMA steps over up.cd (max)
    __shared__ __attribute__((aligned(16))) T dpatch[UPCD > 0 ? NDB * 16 * PSD : 1];
    typename P::Frag rwt[UMB * UKS];
    typename P::Acc rbt[UMB][4];   // the chunk's transposed-convolution bias, per accumulator row
    uint4 rd[NDV];

    const int cin_p = c0 + c1;
    const int64_t plane = (int64_t)H * W;
    const T* xs0 = x0 + (int64_t)bz * plane * c0;
    const T* xs1 = x1 ? x1 + (int64_t)bz * plane * c1 : nullptr;

    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    AccV acc[RPW][NCB];
#pragma unroll
    for (int pb = 0; pb < RPW; ++pb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[pb][cb][r] = 0;

    const int vpp = ck / VE;                   // vectors per pixel in this chunk
    const int cpg = ck / P::GW;                // k-groups per tap
    const int groups = 9 * cpg;
    const int steps = (groups + 3) / 4;
    const int npa = (TH_ + 2) * (TW + 2) * vpp, npw = 9 * TN * vpp;
    uint4 ra[NS][NPA], rw[NS][NPW];
    const int ukn = UPCD > 0 ? up.cd / (4 * P::GW) : 0;   // MFMA steps of the transposed convolution
    // Staging offsets of this thread, the same for every chunk up to the chunk's channel offset
    // (computed once: index arithmetic per chunk would outweigh the chunk's matrix work). Patch
    // vector i: LDS slot plds (or -1 when the thread has no vector i), source offsets poff0 /
    // poff1 within the first / second input part (-1: outside the image, stored as zeros).
    // Weight vector i: LDS slot wlds (-1: none) and offset woff in the packed weights.
    int plds[NPA], wlds[NPW], woff[NPW];
    int64_t poff0[NPA], poff1[NPA];
#pragma unroll
    for (int i = 0; i < NPA; ++i) {
        const int v = threadIdx.x + i * CT;
        plds[i] = -1;
        poff0[i] = poff1[i] = -1;
        if (v < npa) {
            const int px = v / vpp, part = v - px * vpp;
            const int py = px / (TW + 2), pxx = px - py * (TW + 2);
            const int gy = ty0 + py - 1, gx = tx0 + pxx - 1;
            plds[i] = px * PS + part * VE;
            if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
                const int64_t pix = (int64_t)gy * W + gx;
                poff0[i] = pix * c0 + part * VE;
                poff1[i] = pix * c1 + part * VE;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NPW; ++i) {
        const int v = threadIdx.x + i * CT;
        wlds[i] = woff[i] = -1;
        if (v < npw) {
            const int row = v / vpp, part = v - row * vpp;
            const int tap = row / TN, co = row - tap * TN;
            wlds[i] = row * PS + part * VE;
            woff[i] = (tap * cout_p + co0 + co) * cin_p + part * VE;
        }
    }
    auto gload = [&](int k0, uint4 (&ra_)[NPA], uint4 (&rw_)[NPW]) {
        const bool uchunk = UPCD > 0 && k0 >= c0;
        if constexpr (UPCD > 0) {
            if (uchunk) {
                // a U chunk: this wavefront's fragments of the transposed weights (parity wv,
                // channels k0 - c0 + 16 mb + lane % 16, input channels 4 GW ks + GW (lane / 16) ...)
                // and the bias of its accumulator rows
                const T* wt = (const T*)up.wt;
#pragma unroll
                for (int mb = 0; mb < UMB; ++mb)
#pragma unroll
                    for (int ks = 0; ks < UKS; ++ks)
                        if (ks < ukn)
                            rwt[mb * UKS + ks] = P::load(wt + ((int64_t)wv * c1 + (k0 - c0) + mb * 16 + lr) * up.cd +
                                                         ks * 4 * P::GW + lg * P::GW);
#pragma unroll
                for (int mb = 0; mb < UMB; ++mb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) rbt[mb][r] = ((const Acc*)up.bt)[k0 - c0 + mb * 16 + P::row_of(lg, r)];
            }
        }
        // (the fused form stages only the first part from memory)
        const bool first = UPCD > 0 || k0 < c0;
        const T* pbase = first ? xs0 + k0 : xs1 + (k0 - c0);
#pragma unroll
        for (int i = 0; i < NPA; ++i) {
            const int64_t off = first ? poff0[i] : poff1[i];
            ra_[i] = (off >= 0 && !uchunk) ? *(const uint4*)(pbase + off) : uint4{0, 0, 0, 0};
        }
#pragma unroll
        for (int i = 0; i < NPW; ++i) rw_[i] = woff[i] >= 0 ? *(const uint4*)(w + woff[i] + k0) : uint4{0, 0, 0, 0};
    };
    auto lstore = [&](int k0, int st, const uint4 (&ra_)[NPA], const uint4 (&rw_)[NPW]) {
#pragma unroll
        for (int i = 0; i < NPA; ++i)
            if (plds[i] >= 0 && !(UPCD > 0 && k0 >= c0)) *(uint4*)&patch[st * PSZ + plds[i]] = ra_[i];
#pragma unroll
        for (int i = 0; i < NPW; ++i)
            if (wlds[i] >= 0) *(uint4*)&wl[st * WSZ + wlds[i]] = rw_[i];
    };
    const int hd = H / 2, wd = W / 2, dr0 = ty0 / 2 - 1, dc0 = tx0 / 2 - 1;
    if constexpr (UPCD > 0) {
        // the coarse patch, every channel (zero outside the coarse grid)
        const int vpd = up.cd / VE;
        const T* ds = (const T*)up.d + (int64_t)bz * hd * wd * up.cd;
#pragma unroll
        for (int i = 0; i < NDV; ++i) {
            const int v = threadIdx.x + i * CT;
            uint4 val = uint4{0, 0, 0, 0};
            if (v < NDP * vpd) {
                const int px = v / vpd, part = v - px * vpd;
                const int gy = dr0 + px / DC, gx = dc0 + px % DC;
                if (gy >= 0 && gy < hd && gx >= 0 && gx < wd)
                    val = *(const uint4*)(ds + ((int64_t)gy * wd + gx) * up.cd + part * VE);
            }
            rd[i] = val;
        }
    }
    // the epilogue's bias (and fused head weights), fetched with the first chunk
    Acc bpre[NCB][4], hw0[NCB][4], hw1[NCB][4];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = co0 + cb * 16 + P::row_of(lg, r);
            bpre[cb][r] = (bias && !splitp) ? bias[co] : Acc(0);
            hw0[cb][r] = ex.head_w ? P::val(((const T*)ex.head_w)[co]) : Acc(0);
            hw1[cb][r] = ex.head_w ? P::val(((const T*)ex.head_w)[cout_p + co]) : Acc(0);
        }
    const Acc hb0 = ex.head_w ? ((const Acc*)ex.head_b)[0] : Acc(0);
    const Acc hb1 = ex.head_w ? ((const Acc*)ex.head_b)[1] : Acc(0);
    // The matrix-core work of the chunk held in LDS stage stg.
    auto compute = [&](int stg) {
        if (ck == P::CK) {
            conv3_chunk_mma<P, TN, RPW>(acc, &patch[stg * PSZ], &wl[stg * WSZ], wv, lr, lg);
            return;
        }
        for (int sp = 0; sp < steps; ++sp) {
            const int gi = 4 * sp + lg;
            Frag a[NCB], b[RPW];
            if (gi < groups) {
                const int tap = gi / cpg, cg = gi - tap * cpg;
                const int dy = tap / 3, dx = tap - 3 * (tap / 3);
#pragma unroll
                for (int pb = 0; pb < RPW; ++pb)
                    b[pb] = P::load(&patch[stg * PSZ + ((RPW * wv + pb + dy) * (TW + 2) + lr + dx) * PS + cg * P::GW]);
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) a[cb] = P::load(&wl[stg * WSZ + (tap * TN + cb * 16 + lr) * PS + cg * P::GW]);
            } else {
#pragma unroll
                for (int pb = 0; pb < RPW; ++pb) b[pb] = P::zero();
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) a[cb] = P::zero();
            }
#pragma unroll
            for (int pb = 0; pb < RPW; ++pb)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) acc[pb][cb] = P::mma(a[cb], b[pb], acc[pb][cb]);
        }
    };
    // One stage (chunks k0, k0 + ck, ... below kend, at most NS): put the registers in LDS, then
    // refill them with the stage from kpre on (if any) while the matrix cores work on this one.
    auto step = [&](int k0, int kpre) {
        __syncthreads();
#pragma unroll
        for (int st = 0; st < NS; ++st)
            if (k0 + st * ck < kend) lstore(k0 + st * ck, st, ra[st], rw[st]);
        if constexpr (UPCD > 0) {
            if (k0 == kbeg) {
                const int vpd = up.cd / VE;
#pragma unroll
                for (int i = 0; i < NDV; ++i) {
                    const int v = threadIdx.x + i * CT;
                    if (v < NDP * vpd) {
                        const int px = v / vpd, part = v - px * vpd;
                        *(uint4*)&dpatch[px * PSD + part * VE] = rd[i];
                    }
                }
            }
        }
        __syncthreads();
        if constexpr (UPCD > 0) {
            if (k0 >= c0) {
                // U chunk: wavefront wv computes parity (a, b) = (wv / 2, wv % 2) of channels
                // k0 - c0 .. + CK for every coarse pixel, then writes them into the patch
                const int pa = wv >> 1, pb2 = wv & 1;
                // one block of 16 coarse pixels at a time (few live accumulators)
#pragma unroll 1
                for (int nb = 0; nb < NDB; ++nb) {
                    AccV au[UMB];
#pragma unroll
                    for (int mb = 0; mb < UMB; ++mb)
#pragma unroll
                        for (int r = 0; r < 4; ++r) au[mb][r] = 0;
#pragma unroll
                    for (int ks = 0; ks < UKS; ++ks) {
                        if (ks < ukn) {
                            const Frag bf = P::load(&dpatch[(nb * 16 + lr) * PSD + ks * 4 * P::GW + lg * P::GW]);
#pragma unroll
                            for (int mb = 0; mb < UMB; ++mb) au[mb] = P::mma(rwt[mb * UKS + ks], bf, au[mb]);
                        }
                    }
                    const int n = nb * 16 + lr;
                    const int py = 2 * (n / DC) + pa - 1, pxx = 2 * (n % DC) + pb2 - 1;
                    if (n < NDP && py >= 0 && py < TH_ + 2 && pxx >= 0 && pxx < TW + 2) {
                        const int gy = ty0 - 1 + py, gx = tx0 - 1 + pxx;
                        const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
#pragma unroll
                        for (int mb = 0; mb < UMB; ++mb) {
                            Acc t[4];
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                t[r] = in ? au[mb][r] + rbt[mb][r] : Acc(0);
                            store_rows<P>(&patch[(py * (TW + 2) + pxx) * PS + mb * 16 + P::row_of(lg, 0)], t);
                        }
                    }
                }
                __syncthreads();
            }
        }
#pragma unroll
        for (int st = 0; st < NS; ++st)
            if (kpre + st * ck < kend) gload(kpre + st * ck, ra[st], rw[st]);
#pragma unroll
        for (int st = 0; st < NS; ++st)
            if (k0 + st * ck < kend) compute(st);
    };
    gload(kbeg, ra[0], rw[0]);
#pragma unroll
    for (int st = 1; st < NS; ++st)
        if (kbeg + st * ck < kend) gload(kbeg + st * ck, ra[st], rw[st]);
    asm volatile("" ::: "memory");   // keep the loads above the test
    if (skipped) return;             // uniform over the block
    for (int k0 = kbeg; k0 < kend; k0 += NS * ck) step(k0, k0 + NS * ck);


    const int gx = tx0 + lr;
    if (splitp) {
        Acc* sp = splitp + (int64_t)bz * plane * cout_p;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int pb = 0; pb < RPW; ++pb) {
                const int gy = ty0 + RPW * wv + pb;
                if (gy < H && gx < W) {
                    Acc* dst = sp + ((int64_t)gy * W + gx) * cout_p + co0 + cb * 16;
#pragma unroll
                    for (int r = 0; r < 4; ++r) dst[P::row_of(lg, r)] = acc[pb][cb][r];
                }
            }
        return;
    }
    if (ex.head_w) {   // fused 1x1 head over all cout_p = TN channels of the pixel
        Acc o0[RPW], o1[RPW];
#pragma unroll
        for (int pb = 0; pb < RPW; ++pb) o0[pb] = o1[pb] = Acc(0);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const Acc w0 = hw0[cb][r], w1 = hw1[cb][r], bc = bpre[cb][r];
#pragma unroll
                for (int pb = 0; pb < RPW; ++pb) {
                    Acc t = acc[pb][cb][r] + bc;
                    if (relu) t = t > Acc(0) ? t : Acc(0);
                    t = P::val(P::cvt(t));
                    o0[pb] += t * w0;
                    o1[pb] += t * w1;
                }
            }
        const double sfac = ex.head_fixed_s > 0 ? ex.head_fixed_s : ex.head_sc[0];
#pragma unroll
        for (int pb = 0; pb < RPW; ++pb) {
            Acc a0 = o0[pb], a1 = o1[pb];
            a0 += __shfl_xor(a0, 16, 64);
            a1 += __shfl_xor(a1, 16, 64);
            a0 += __shfl_xor(a0, 32, 64);
            a1 += __shfl_xor(a1, 32, 64);
            const int gy = ty0 + RPW * wv + pb;
            if (lg == 0 && gy < ex.head_nyt && gx < ex.head_nxt) {
                const double2 zv{sfac * (double)(hb0 + a0), sfac * (double)(hb1 + a1)};
                const int64_t zi = (int64_t)gy * ex.head_nxt + gx;
                if (ex.head_c128) ((double2*)ex.head_z)[zi] = zv;
                else ((float2*)ex.head_z)[zi] = from_d2<float2>(zv);
            }
        }
        return;
    }
    // epilogue: register r of a lane holds output channel co0 + 16 cb + row_of(lg, r) of pixel
    // (ty0 + RPW wv + pb, tx0 + lr). Channels below ex.split go to y (ex.split channels per pixel),
    // the others to ex.y1_; ex.mask0_ / ex.mask1_ (same layouts) zero the entries whose mask is <= 0.
    const int split = ex.split > 0 ? ex.split : cout_p;
    const bool second = co0 >= split;
    const int cst = second ? cout_p - split : split;          // channels per pixel of this output
    T* ys = (second ? (T*)ex.y1_ : y) + (int64_t)bz * plane * cst;
    const T* ms = (const T*)(second ? ex.mask1_ : ex.mask0_);
    if (ms) ms += (int64_t)bz * plane * cst;
    const int cbase = second ? co0 - split : co0;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int co = co0 + cb * 16;
        const int cl = cbase + cb * 16;
        Acc v[RPW][4];
#pragma unroll
        for (int pb = 0; pb < RPW; ++pb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Acc t = acc[pb][cb][r] + bpre[cb][r];
                if (relu) t = t > Acc(0) ? t : Acc(0);
                v[pb][r] = t;
            }
#pragma unroll
        for (int pb = 0; pb < RPW; ++pb) {
            const int gy = ty0 + RPW * wv + pb;
            if (gy < H && gx < W) {
                const int64_t off = ((int64_t)gy * W + gx) * cst + cl;
                Acc t[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    t[r] = v[pb][r];
                    if (ms && !(P::val(ms[off + P::row_of(lg, r)]) > Acc(0))) t[r] = Acc(0);
                }
                store_rows<P>(ys + off + P::row_of(lg, 0), t);
            }
        }
        if (POOL) {
            T* ps = ypool + (int64_t)bz * (plane / 4) * cout_p;
#pragma unroll
            for (int pp = 0; pp < RPW; pp += 2) {
                Acc q[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    Acc s = v[pp][r] + v[pp + 1][r];
                    s += __shfl_xor(s, 1, 64);
                    q[r] = Acc(0.25) * s;
                }
                const int gy = ty0 + RPW * wv + pp;
                if ((lr & 1) == 0 && gy < H && gx < W)
                    store_rows<P>(ps + ((int64_t)(gy / 2) * (W / 2) + gx / 2) * cout_p + co + P::row_of(lg, 0), q);
            }
        }
    }
}

// Split-K reduction and epilogue: y = act(sum_s part[s] + b) (+ pooled copy). One thread per
// output channel of one pixel (or of one 2 x 2 block when pooling).
template <class P, bool POOL>
__global__ void k_splitk_epilogue(const typename P::Acc* __restrict__ part, int nsplit, int64_t sstride,
                                  const typename P::Acc* __restrict__ bias, typename P::T* __restrict__ y,
                                  typename P::T* __restrict__ ypool, int H, int W, int cout_p, int batch, int relu,
                                  const int* __restrict__ skip) {
    using Acc = typename P::Acc;
    if (skip && *skip) return;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = (int)(idx % cout_p);
    const int64_t q = idx / cout_p;
    if (!POOL) {
        if (q >= (int64_t)batch * H * W) return;
        Acc s = bias[c];
        for (int k = 0; k < nsplit; ++k) s += part[k * sstride + q * cout_p + c];
        if (relu) s = s > Acc(0) ? s : Acc(0);
        y[q * cout_p + c] = P::cvt(s);
    } else {
        const int Hh = H / 2, Wh = W / 2;
        if (q >= (int64_t)batch * Hh * Wh) return;
        const int b = (int)(q / ((int64_t)Hh * Wh));
        const int64_t r = q - (int64_t)b * Hh * Wh;
        const int py = (int)(r / Wh), px = (int)(r % Wh);
        Acc pool = 0;
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int64_t pix = (int64_t)b * H * W + (int64_t)(2 * py + dy) * W + 2 * px + dx;
                Acc s = bias[c];
                for (int k = 0; k < nsplit; ++k) s += part[k * sstride + pix * cout_p + c];
                if (relu) s = s > Acc(0) ? s : Acc(0);
                y[pix * cout_p + c] = P::cvt(s);
                pool += s;
            }
        ypool[q * cout_p + c] = P::cvt(Acc(0.25) * pool);
    }
}

// grid: x = column tiles, y = row tiles, z = (sample, channel block, K split)
template <class P, int TN, bool POOL, int RPW, int NS = 1>
__global__ __launch_bounds__(CT) void k_conv3(const typename P::T* __restrict__ x0, int c0,
                                              const typename P::T* __restrict__ x1, int c1,
                                              const typename P::T* __restrict__ w,
                                              const typename P::Acc* __restrict__ bias,
                                              typename P::T* __restrict__ y, int cout_p,
                                              typename P::T* __restrict__ ypool, int H, int W, int relu, int ck,
                                              const int* __restrict__ skip, Conv3Out ex, int nsplit,
                                              typename P::Acc* __restrict__ splitp, int64_t sstride) {
    // logical order: channel block fastest, then K split, column tile, row tile, sample
    const int ncb_tot = cout_p / TN;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    int v = xcd_linear(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nblk);
    const int cbi = v % ncb_tot;
    v /= ncb_tot;
    const int zs = v % nsplit;
    v /= nsplit;
    const int txi = v % gridDim.x;
    v /= gridDim.x;
    const int tyi = v % gridDim.y;
    const int bz = v / gridDim.y;                // sample
    const int co0 = cbi * TN;
    const int cin_p = c0 + c1;
    const int nch = cin_p / ck;
    const int kb = (nch * zs / nsplit) * ck, ke = (nch * (zs + 1) / nsplit) * ck;
    conv3_tile<P, TN, POOL, RPW, 0, NS>(x0, c0, x1, c1, w, bias, y, cout_p, ypool, H, W, relu, ck, ex, bz, co0,
                                 tyi * 4 * RPW, txi * TW, kb, ke, splitp ? splitp + zs * sstride : nullptr, UpIn(),
                                 skip);
}

// Weight-stationary 3x3 convolution for layers with few input channels on large grids, with
// loader and compute wavefronts. A block of 8 wavefronts keeps the weights of its TN output
// channels for all WCH chunks (9 x TN x cin_p, the whole input) in LDS, loaded once, and runs tpb
// consecutive pixel tiles with them (row-major tile order of the sample). Wavefronts 4-7 only
// load: they hold the patches (all chunks) of the next K tiles in K register sets and move one
// tile per step into a double-buffered LDS patch; wavefronts 0-3 only compute and store: per step
// they run the matrix cores on the tile staged in the previous step and write its outputs. Each
// wavefront's memory counter then tracks loads only or stores only, so a loader waits for its
// oldest tile alone while K - 1 tiles of loads stay in flight. One barrier per step. Every output
// is accumulated chunk by chunk and tap by tap as in conv3_tile (same result bits as the other
// variants). Plain epilogue: bias, ReLU, optional 2 x 2 average pool.
// With HEAD (TN == cout_p) the epilogue is the fused 1x1 head of conv3_tile instead (ex.head_*).
constexpr int WS_THREADS = 2 * CT;
// One block: output channels [co0, co0 + TN) of tiles [t_beg, t_end) of one sample (xs0, xs1, ys,
// yps already point at the sample; tiles row-major over the image, TW wide and 4 RPW high).
template <class P, int TN, bool POOL, int RPW, int WCH, int K, bool HEAD, bool SMALL = false, bool MASKED = false>
__device__ __forceinline__ void conv3_ws_body(const typename P::T* __restrict__ xs0, int c0,
                                              const typename P::T* __restrict__ xs1, int c1,
                                              const typename P::T* __restrict__ w,
                                              const typename P::Acc* __restrict__ bias,
                                              typename P::T* __restrict__ ys, int cout_p,
                                              typename P::T* __restrict__ yps, int H, int W, int relu, int co0,
                                              int t_beg, int t_end, int skipped, const Conv3Out& ex) {
    using T = typename P::T;
    using Acc = typename P::Acc;
    using AccV = typename P::AccV;
    static_assert(!HEAD || !POOL, "the fused head has no pooled output");
    static_assert(!SMALL || WCH == 1, "an input of one k-group per tap is one chunk");
    // MASKED: conv3_tile's split / masked epilogue (ex.split, ex.y1_, ex.mask0_, ex.mask1_, already
    // at the sample) and an optional bias, for the data gradient of training (BF16: a lane's 4
    // registers are 4 consecutive channels, whose mask entries are one 8-byte load)
    static_assert(!MASKED || (!HEAD && !POOL && std::is_same<P, PolBF16>::value),
                  "the masked epilogue: BF16, no head or pooled output");
    constexpr int TH_ = 4 * RPW;
    constexpr int PS = pix_stride<P>();
    constexpr int VE = 16 / sizeof(T);
    constexpr int NCB = TN / 16;
    constexpr int VPP = SMALL ? 1 : P::CK / VE;           // vectors per pixel of a chunk
    constexpr int PSZ = (TH_ + 2) * (TW + 2) * PS, WSZ = 9 * TN * PS;
    constexpr int NPV = (TH_ + 2) * (TW + 2) * VPP;       // patch vectors per chunk
    constexpr int NPA = (NPV + CT - 1) / CT;              // per loader thread
    constexpr int NPW = (9 * TN * VPP + WS_THREADS - 1) / WS_THREADS;   // weight vectors per thread
    __shared__ __attribute__((aligned(16))) T patch[2 * WCH * PSZ];
    __shared__ __attribute__((aligned(16))) T wl[WCH * WSZ];

    const int cin_p = c0 + c1;
    const int nch = SMALL ? 1 : cin_p / P::CK;   // <= WCH (checked on the host)
    const int ntx = (W + TW - 1) / TW;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool loader = wv >= 4;
    const int lt = threadIdx.x - CT;   // loader thread index (loaders only)
    const int lr = lane & 15, lg = lane >> 4;

    // weights of all chunks (every wavefront): into registers together, then into LDS
    {
        uint4 rw[WCH][NPW];
#pragma unroll
        for (int c = 0; c < WCH; ++c)
#pragma unroll
            for (int i = 0; i < NPW; ++i) {
                const int vv = threadIdx.x + i * WS_THREADS;
                rw[c][i] = uint4{0, 0, 0, 0};
                if (c < nch && vv < 9 * TN * VPP) {
                    const int row = vv / VPP, part = vv - row * VPP;
                    const int tap = row / TN, co = row - tap * TN;
                    rw[c][i] = *(const uint4*)(w + (int64_t)(tap * cout_p + co0 + co) * cin_p + c * P::CK + part * VE);
                }
            }
#pragma unroll
        for (int c = 0; c < WCH; ++c)
#pragma unroll
            for (int i = 0; i < NPW; ++i) {
                const int vv = threadIdx.x + i * WS_THREADS;
                if (c < nch && vv < 9 * TN * VPP) {
                    const int row = vv / VPP, part = vv - row * VPP;
                    *(uint4*)&wl[c * WSZ + row * PS + part * VE] = rw[c][i];
                }
            }
    }
    // loader: the patches of all chunks of tile t into ra_. Every lane loads unconditionally (from
    // pixel 0 where its pixel is outside the image), so that the number of loads in flight does not
    // depend on the data; ok_ marks the vectors inside, and lstore writes zeros for the others.
    auto gload = [&](int t, uint4 (&ra_)[WCH][NPA], uint32_t& ok_) {
        const int ty0 = (t / ntx) * TH_, tx0 = (t % ntx) * TW;
        ok_ = 0;
#pragma unroll
        for (int i = 0; i < NPA; ++i) {
            const int vv = min(lt + i * CT, NPV - 1);
            const int px = vv / VPP;
            const int part = vv - px * VPP;
            const int py = px / (TW + 2), pxx = px - py * (TW + 2);
            const int gy = ty0 + py - 1, gx = tx0 + pxx - 1;
            const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
            const int64_t pix = in ? (int64_t)gy * W + gx : 0;
            ok_ |= (in ? 1u : 0u) << i;
#pragma unroll
            for (int c = 0; c < WCH; ++c) {
                const int k0 = c * P::CK;
                const T* src = k0 < c0 ? xs0 + pix * c0 + k0 : xs1 + pix * c1 + (k0 - c0);
                ra_[c][i] = *(const uint4*)(src + part * VE);
            }
        }
    };
    // loader: a register set into LDS patch buffer b
    auto lstore = [&](int b, const uint4 (&ra_)[WCH][NPA], uint32_t ok_) {
#pragma unroll
        for (int i = 0; i < NPA; ++i) {
            const int vv = lt + i * CT;
            if (vv < NPV) {
                const int px = vv / VPP, part = vv - px * VPP;
                const bool in = (ok_ >> i) & 1u;
#pragma unroll
                for (int c = 0; c < WCH; ++c)
                    *(uint4*)&patch[(b * WCH + c) * PSZ + px * PS + part * VE] = in ? ra_[c][i] : uint4{0, 0, 0, 0};
            }
        }
    };
    // loader set u holds tile t_beg + u + K j for j = 0, 1, ...
    uint4 ra[K][WCH][NPA];
    uint32_t ok[K];
    if (loader) {
#pragma unroll
        for (int u = 0; u < K; ++u) gload(min(t_beg + u, t_end - 1), ra[u], ok[u]);
    }
    asm volatile("" ::: "memory");       // keep the loads above the test
    if (skipped) return;                 // uniform over the block
    if (loader) lstore(0, ra[0], ok[0]);   // tile t_beg into buffer 0
    __syncthreads();

    // compute wavefronts: tile t from LDS buffer b, outputs to memory
    Acc bpre[NCB][4], hw0[NCB][4], hw1[NCB][4];
    Acc hb0 = Acc(0), hb1 = Acc(0);
    auto compute = [&](int t, int b) {
        // (MASKED) the mask entries of this tile's outputs, loaded before the matrix-core work
        uint2 mk[MASKED ? RPW : 1][MASKED ? NCB : 1];
        if constexpr (MASKED) {
            const int split = ex.split > 0 ? ex.split : cout_p;
            const bool second = co0 >= split;
            const int cst = second ? cout_p - split : split;
            const T* ms = (const T*)(second ? ex.mask1_ : ex.mask0_);
            const int cbase = second ? co0 - split : co0;
            const int ty0m = (t / ntx) * TH_, gxm = (t % ntx) * TW + lr;
#pragma unroll
            for (int pb = 0; pb < RPW; ++pb)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    const int gy = ty0m + RPW * wv + pb;
                    mk[pb][cb] = uint2{0x3f803f80u, 0x3f803f80u};   // 1.0 in every entry: kept
                    if (ms && gy < H && gxm < W)
                        mk[pb][cb] = *(const uint2*)(ms + ((int64_t)gy * W + gxm) * cst + cbase + cb * 16 +
                                                     P::row_of(lg, 0));
                }
        }
        AccV acc[RPW][NCB];
#pragma unroll
        for (int pb = 0; pb < RPW; ++pb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[pb][cb][r] = 0;
#pragma unroll
        for (int c = 0; c < WCH; ++c)
            if (c < nch) {
                if constexpr (SMALL) conv3_group_mma<P, TN, RPW>(acc, &patch[(b * WCH + c) * PSZ], &wl[c * WSZ], wv, lr, lg);
                else conv3_chunk_mma<P, TN, RPW>(acc, &patch[(b * WCH + c) * PSZ], &wl[c * WSZ], wv, lr, lg);
            }
        // register r of a lane holds output channel co0 + 16 cb + row_of(lg, r) of pixel
        // (ty0 + RPW wv + pb, tx0 + lr)
        const int ty0 = (t / ntx) * TH_, tx0 = (t % ntx) * TW;
        const int gx = tx0 + lr;
        if constexpr (HEAD) {   // as conv3_tile's fused head: rounded activations, then the 1x1 head
            Acc o0[RPW], o1[RPW];
#pragma unroll
            for (int pb = 0; pb < RPW; ++pb) o0[pb] = o1[pb] = Acc(0);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const Acc w0 = hw0[cb][r], w1 = hw1[cb][r], bc = bpre[cb][r];
#pragma unroll
                    for (int pb = 0; pb < RPW; ++pb) {
                        Acc q = acc[pb][cb][r] + bc;
                        if (relu) q = q > Acc(0) ? q : Acc(0);
                        q = P::val(P::cvt(q));
                        o0[pb] += q * w0;
                        o1[pb] += q * w1;
                    }
                }
            const double sfac = ex.head_fixed_s > 0 ? ex.head_fixed_s : ex.head_sc[0];
#pragma unroll
            for (int pb = 0; pb < RPW; ++pb) {
                Acc a0 = o0[pb], a1 = o1[pb];
                a0 += __shfl_xor(a0, 16, 64);
                a1 += __shfl_xor(a1, 16, 64);
                a0 += __shfl_xor(a0, 32, 64);
                a1 += __shfl_xor(a1, 32, 64);
                const int gy = ty0 + RPW * wv + pb;
                if (lg == 0 && gy < ex.head_nyt && gx < ex.head_nxt) {
                    const double2 zv{sfac * (double)(hb0 + a0), sfac * (double)(hb1 + a1)};
                    const int64_t zi = (int64_t)gy * ex.head_nxt + gx;
                    if (ex.head_c128) ((double2*)ex.head_z)[zi] = zv;
                    else ((float2*)ex.head_z)[zi] = from_d2<float2>(zv);
                }
            }
            return;
        }
        if constexpr (MASKED) {   // as conv3_tile's epilogue with an output split and masks
            const int split = ex.split > 0 ? ex.split : cout_p;
            const bool second = co0 >= split;
            const int cst = second ? cout_p - split : split;   // channels per pixel of this output
            T* yb = second ? (T*)ex.y1_ : ys;
            const int cbase = second ? co0 - split : co0;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const int cl = cbase + cb * 16;
#pragma unroll
                for (int pb = 0; pb < RPW; ++pb) {
                    const int gy = ty0 + RPW * wv + pb;
                    if (gy < H && gx < W) {
                        const int64_t off = ((int64_t)gy * W + gx) * cst + cl;
                        Acc q[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            q[r] = acc[pb][cb][r] + bpre[cb][r];
                            if (relu) q[r] = q[r] > Acc(0) ? q[r] : Acc(0);
                            const uint32_t mw = r < 2 ? mk[pb][cb].x : mk[pb][cb].y;
                            const T m = (T)((mw >> (16 * (r & 1))) & 0xffffu);
                            if (!(P::val(m) > Acc(0))) q[r] = Acc(0);
                        }
                        store_rows<P>(yb + off + P::row_of(lg, 0), q);
                    }
                }
            }
            return;
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int co = co0 + cb * 16;
            Acc vv[RPW][4];
#pragma unroll
            for (int pb = 0; pb < RPW; ++pb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    Acc q = acc[pb][cb][r] + bpre[cb][r];
                    if (relu) q = q > Acc(0) ? q : Acc(0);
                    vv[pb][r] = q;
                }
#pragma unroll
            for (int pb = 0; pb < RPW; ++pb) {
                const int gy = ty0 + RPW * wv + pb;
                if (gy < H && gx < W) store_rows<P>(ys + ((int64_t)gy * W + gx) * cout_p + co + P::row_of(lg, 0), vv[pb]);
            }
            if (POOL) {
                T* ps = yps;
#pragma unroll
                for (int pp = 0; pp < RPW; pp += 2) {
                    Acc q[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        Acc sm = vv[pp][r] + vv[pp + 1][r];
                        sm += __shfl_xor(sm, 1, 64);
                        q[r] = Acc(0.25) * sm;
                    }
                    const int gy = ty0 + RPW * wv + pp;
                    if ((lr & 1) == 0 && gy < H && gx < W)
                        store_rows<P>(ps + ((int64_t)(gy / 2) * (W / 2) + gx / 2) * cout_p + co + P::row_of(lg, 0), q);
                }
            }
        }
    };
    // Step i (tile t = t_beg + i), one barrier each: the compute wavefronts work on buffer i % 2
    // while the loaders move tile t + 1 (register set (i + 1) % K) into buffer (i + 1) % 2 and
    // refill set i % K with tile t + K. The two roles run separate loops with the same number of
    // barriers (the role is uniform per wavefront), so that each role's code holds only its own
    // kind of memory operation and its waits count only those.
    if (loader) {
        for (int t0 = t_beg; t0 < t_end; t0 += K) {
#pragma unroll
            for (int u = 0; u < K; ++u) {
                const int t = t0 + u;
                if (t < t_end) {
                    const int b = (t - t_beg) & 1;
                    if (t + 1 < t_end) lstore(b ^ 1, ra[(u + 1) % K], ok[(u + 1) % K]);
                    // (past the group's last tile the set reloads that tile: the same number of
                    // loads on every path)
                    gload(min(t + K, t_end - 1), ra[u], ok[u]);
                    __syncthreads();
                }
            }
        }
    } else {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = co0 + cb * 16 + P::row_of(lg, r);
                if constexpr (MASKED) bpre[cb][r] = bias ? bias[co] : Acc(0);
                else bpre[cb][r] = bias[co];
                if constexpr (HEAD) {
                    hw0[cb][r] = P::val(((const T*)ex.head_w)[co]);
                    hw1[cb][r] = P::val(((const T*)ex.head_w)[cout_p + co]);
                }
            }
        if constexpr (HEAD) {
            hb0 = ((const Acc*)ex.head_b)[0];
            hb1 = ((const Acc*)ex.head_b)[1];
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): bias (and head) in registers before the loop
        for (int t = t_beg; t < t_end; ++t) {
            compute(t, (t - t_beg) & 1);
            __syncthreads();
        }
    }
}

// grid: x = tile groups (tpb tiles each), y = channel blocks, z = samples; logical block order:
// channel block fastest, then tile group, then sample.
template <class P, int TN, bool POOL, int RPW, int WCH, int K>
__global__ __launch_bounds__(WS_THREADS) void k_conv3_ws(const typename P::T* __restrict__ x0, int c0,
                                                         const typename P::T* __restrict__ x1, int c1,
                                                         const typename P::T* __restrict__ w,
                                                         const typename P::Acc* __restrict__ bias,
                                                         typename P::T* __restrict__ y, int cout_p,
                                                         typename P::T* __restrict__ ypool, int H, int W, int relu,
                                                         int tpb, const int* __restrict__ skip) {
    const int skipped = skip ? *skip : 0;   // tested once the first loads are in flight
    const int ncb_tot = gridDim.y;
    const int ngrp = gridDim.x;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    int v = xcd_linear(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nblk);
    const int cbi = v % ncb_tot;
    v /= ncb_tot;
    const int grp = v % ngrp;
    const int bz = v / ngrp;
    const int ntiles = ((W + TW - 1) / TW) * ((H + 4 * RPW - 1) / (4 * RPW));
    const int t_beg = grp * tpb, t_end = min(ntiles, t_beg + tpb);
    const int64_t plane = (int64_t)H * W;
    conv3_ws_body<P, TN, POOL, RPW, WCH, K, false>(
        x0 + (int64_t)bz * plane * c0, c0, x1 ? x1 + (int64_t)bz * plane * c1 : nullptr, c1, w, bias,
        y + (int64_t)bz * plane * cout_p, cout_p, POOL ? ypool + (int64_t)bz * (plane / 4) * cout_p : nullptr, H, W,
        relu, cbi * TN, t_beg, t_end, skipped, Conv3Out());
}

// The same for an input of one k-group per tap (conv3_ws_small): no pooled output.
template <class P, int TN, int RPW, int K>
__global__ __launch_bounds__(WS_THREADS) void k_conv3_ws8(const typename P::T* __restrict__ x0, int c0,
                                                          const typename P::T* __restrict__ w,
                                                          const typename P::Acc* __restrict__ bias,
                                                          typename P::T* __restrict__ y, int cout_p, int H, int W,
                                                          int relu, int tpb, const int* __restrict__ skip) {
    const int skipped = skip ? *skip : 0;   // tested once the first loads are in flight
    const int ncb_tot = gridDim.y;
    const int ngrp = gridDim.x;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    int v = xcd_linear(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nblk);
    const int cbi = v % ncb_tot;
    v /= ncb_tot;
    const int grp = v % ngrp;
    const int bz = v / ngrp;
    const int ntiles = ((W + TW - 1) / TW) * ((H + 4 * RPW - 1) / (4 * RPW));
    const int t_beg = grp * tpb, t_end = min(ntiles, t_beg + tpb);
    const int64_t plane = (int64_t)H * W;
    const typename P::T* xs = x0 + (int64_t)bz * plane * c0;
    // (the second input part is empty; xs stands in for its pointer, which is never read)
    conv3_ws_body<P, TN, false, RPW, 1, K, false, true>(xs, c0, xs, 0, w, bias,
                                                        y + (int64_t)bz * plane * cout_p, cout_p, nullptr, H, W, relu,
                                                        cbi * TN, t_beg, t_end, skipped, Conv3Out());
}

// The data gradient of training in the weight-stationary form (one input x0 of c0 channels, no
// bias or activation): output channels below split go to y0 (split per pixel), the others to y1;
// an entry whose mask entry (mask0 / mask1, the same layouts) is <= 0 is zero.
template <class P, int TN, int RPW, int WCH, int K>
__global__ __launch_bounds__(WS_THREADS) void k_conv3_ws_dgrad(const typename P::T* __restrict__ x0, int c0,
                                                               const typename P::T* __restrict__ w,
                                                               typename P::T* __restrict__ y0, int cout_p, int H, int W,
                                                               int tpb, int split, typename P::T* __restrict__ y1,
                                                               const typename P::T* __restrict__ mask0,
                                                               const typename P::T* __restrict__ mask1) {
    const int ncb_tot = gridDim.y;
    const int ngrp = gridDim.x;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    int v = xcd_linear(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nblk);
    const int cbi = v % ncb_tot;
    v /= ncb_tot;
    const int grp = v % ngrp;
    const int bz = v / ngrp;
    const int ntiles = ((W + TW - 1) / TW) * ((H + 4 * RPW - 1) / (4 * RPW));
    const int t_beg = grp * tpb, t_end = min(ntiles, t_beg + tpb);
    const int64_t plane = (int64_t)H * W;
    const int s0 = split > 0 ? split : cout_p, s1 = cout_p - s0;
    Conv3Out ex;
    ex.split = split;
    ex.y1_ = y1 ? y1 + (int64_t)bz * plane * s1 : nullptr;
    ex.mask0_ = mask0 ? mask0 + (int64_t)bz * plane * s0 : nullptr;
    ex.mask1_ = mask1 ? mask1 + (int64_t)bz * plane * s1 : nullptr;
    const typename P::T* xs = x0 + (int64_t)bz * plane * c0;
    // (no second input part; xs stands in for its pointer, which is never read)
    conv3_ws_body<P, TN, false, RPW, WCH, K, false, false, true>(xs, c0, xs, 0, w, nullptr,
                                                                 y0 + (int64_t)bz * plane * s0, cout_p, nullptr, H,
                                                                 W, 0, cbi * TN, t_beg, t_end, 0, ex);
}

// Ragged batch, weight-stationary form: job = (system, first output channel, first tile, end
// tile) in the fields (sys, c0, ty0, tx0); with HEAD the fused 1x1 head writes column col of the
// system's z (LayerIO head fields) instead of y.
template <class P, int TN, bool POOL, int RPW, int WCH, int K, bool HEAD, bool SMALL>
__global__ __launch_bounds__(WS_THREADS) void k_conv3_ws_jobs(const TileJob* __restrict__ jobs,
                                                              const LayerIO* __restrict__ io,
                                                              const typename P::T* __restrict__ w,
                                                              const typename P::Acc* __restrict__ bias, int c0, int c1,
                                                              int cout_p, const typename P::T* __restrict__ head_w,
                                                              const typename P::Acc* __restrict__ head_b, int col,
                                                              int c128) {
    const TileJob jb = jobs[xcd_linear(blockIdx.x, gridDim.x)];
    const LayerIO d = io[jb.sys];
    if (d.stop && *d.stop) return;
    Conv3Out ex;
    if constexpr (HEAD) {
        ex.head_w = head_w;
        ex.head_b = head_b;
        ex.head_c128 = c128;
        ex.head_z = c128 ? (void*)((double2*)d.z + (int64_t)col * d.zld) : (void*)((float2*)d.z + (int64_t)col * d.zld);
        ex.head_nxt = d.nxt;
        ex.head_nyt = d.nyt;
        ex.head_sc = d.sc;
    }
    conv3_ws_body<P, TN, POOL, RPW, WCH, K, HEAD, SMALL>((const typename P::T*)d.x0, c0, (const typename P::T*)d.x1, c1, w,
                                                  bias, (typename P::T*)d.y, cout_p, (typename P::T*)d.ypool, d.H,
                                                  d.W, 1, jb.c0, jb.ty0, jb.tx0, 0, ex);
}

// Decoder 3x3 convolution with the transposed convolution of the coarser level fused in (UpIn).
// grid: x = column tiles, y = row tiles, z = (sample, channel block)
template <class P, int TN, int RPW, int UPCD>
__global__ __launch_bounds__(CT) void k_conv3_up(const typename P::T* __restrict__ x0, int c0, UpIn up, int c1,
                                                 const typename P::T* __restrict__ w,
                                                 const typename P::Acc* __restrict__ bias,
                                                 typename P::T* __restrict__ y, int cout_p, int H, int W,
                                                 const int* __restrict__ skip) {
    const int ncb_tot = cout_p / TN;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    int v = xcd_linear(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nblk);
    const int cbi = v % ncb_tot;
    v /= ncb_tot;
    const int txi = v % gridDim.x;
    v /= gridDim.x;
    const int tyi = v % gridDim.y;
    const int bz = v / gridDim.y;
    conv3_tile<P, TN, false, RPW, UPCD>(x0, c0, nullptr, c1, w, bias, y, cout_p, nullptr, H, W, 1, P::CK, Conv3Out(),
                                        bz, cbi * TN, tyi * 4 * RPW, txi * TW, 0, c0 + c1, nullptr, up, skip);
}

// Ragged batch: block b runs job jobs[b] = (system, tile, channel block) with the system's tensors.
template <class P, int TN, bool POOL, int RPW>
__global__ __launch_bounds__(CT) void k_conv3_jobs(const TileJob* __restrict__ jobs, const LayerIO* __restrict__ io,
                                                   const typename P::T* __restrict__ w,
                                                   const typename P::Acc* __restrict__ bias, int c0, int c1,
                                                   int cout_p, int relu, int ck) {
    const TileJob jb = jobs[xcd_linear(blockIdx.x, gridDim.x)];
    const LayerIO d = io[jb.sys];
    if (d.stop && *d.stop) return;
    conv3_tile<P, TN, POOL, RPW>((const typename P::T*)d.x0, c0, (const typename P::T*)d.x1, c1, w, bias,
                               (typename P::T*)d.y, cout_p, (typename P::T*)d.ypool, d.H, d.W, relu, ck, Conv3Out(),
                               0, jb.c0, jb.ty0, jb.tx0, 0, c0 + c1, nullptr);
}

// Last 3x3 layer of a ragged batch with the 1x1 head in its epilogue: TN == cout_p, so one
// block holds every output channel of its pixels; z gets column col of the system's vectors.
template <class P, int TN>
__global__ __launch_bounds__(CT) void k_conv3_jobs_head(const TileJob* __restrict__ jobs,
                                                        const LayerIO* __restrict__ io,
                                                        const typename P::T* __restrict__ w,
                                                        const typename P::Acc* __restrict__ bias, int c0, int c1,
                                                        int ck, const typename P::T* __restrict__ head_w,
                                                        const typename P::Acc* __restrict__ head_b, int col,
                                                        int c128) {
    const TileJob jb = jobs[xcd_linear(blockIdx.x, gridDim.x)];
    const LayerIO d = io[jb.sys];
    if (d.stop && *d.stop) return;
    Conv3Out ex;
    ex.head_w = head_w;
    ex.head_b = head_b;
    ex.head_c128 = c128;
    ex.head_z = c128 ? (void*)((double2*)d.z + (int64_t)col * d.zld) : (void*)((float2*)d.z + (int64_t)col * d.zld);
    ex.head_nxt = d.nxt;
    ex.head_nyt = d.nyt;
    ex.head_sc = d.sc;
    conv3_tile<P, TN, false, 2>((const typename P::T*)d.x0, c0, (const typename P::T*)d.x1, c1, w, bias, nullptr,
                                TN, nullptr, d.H, d.W, 1, ck, ex, 0, 0, jb.ty0, jb.tx0, 0, c0 + c1, nullptr);
}

// 2x2 stride-2 transposed convolution: a GEMM per input pixel with M = 4 x
// output channels (tap a, b and channel), N = 16 input pixels per wave, K = input
// channels. Block: 64 input pixels of one row (4 waves x 16) and TN channels.
template <class P>
constexpr int convT2_ksmax() { return 4 * P::CK; }   // input channels per LDS stage (at most)

// One block: output channels [co0, co0 + TN) of the 4 parities for the 64 input pixels
// (iy, ix0 .. ix0 + 63) of sample bz. Input channels go in stages of ks (<= 4 CK); the next
// stage is loaded into registers while the matrix cores work on the current one, and a stage of
// whole steps runs an unrolled step schedule.
template <class P, int TN>
__device__ __forceinline__ void convT2_tile(const typename P::T* __restrict__ x, int cin_p,
                                            const typename P::T* __restrict__ w,
                                            const typename P::Acc* __restrict__ bias,
                                            typename P::T* __restrict__ y, int cout_p, int H, int W, int ks, int bz,
                                            int co0, int iy, int ix0, const int* __restrict__ skip = nullptr) {
    using T = typename P::T;
    using Acc = typename P::Acc;
    using AccV = typename P::AccV;
    using Frag = typename P::Frag;
    const int skipped = skip ? *skip : 0;   // tested once the first loads are in flight
    constexpr int KSM = convT2_ksmax<P>();
    constexpr int PS = KSM + 16 / (int)sizeof(T);
    constexpr int VE = 16 / sizeof(T);
    constexpr int NCB = TN / 16;
    constexpr int NXV = (64 * KSM / VE + CT - 1) / CT;
    constexpr int NWV = (4 * TN * KSM / VE + CT - 1) / CT;
    __shared__ __attribute__((aligned(16))) T xin[64 * PS];
    __shared__ __attribute__((aligned(16))) T wl[4 * TN * PS];
    const int64_t plane = (int64_t)H * W;
    const T* xs = x + (int64_t)bz * plane * cin_p;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    AccV acc[4][NCB];
#pragma unroll
    for (int ab = 0; ab < 4; ++ab)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[ab][cb][r] = 0;
    const int vpp = ks / VE;
    const int nxv = 64 * vpp, nwv = 4 * TN * vpp;
    uint4 rx[NXV], rw[NWV];
    auto gload = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NXV; ++i) {
            const int v = threadIdx.x + i * CT;
            uint4 val = uint4{0, 0, 0, 0};
            if (v < nxv) {
                const int px = v / vpp, part = v - px * vpp;
                const int gx = ix0 + px;
                if (gx < W) val = *(const uint4*)(xs + ((int64_t)iy * W + gx) * cin_p + k0 + part * VE);
            }
            rx[i] = val;
        }
#pragma unroll
        for (int i = 0; i < NWV; ++i) {
            const int v = threadIdx.x + i * CT;
            uint4 val = uint4{0, 0, 0, 0};
            if (v < nwv) {
                const int row = v / vpp, part = v - row * vpp;
                const int ab = row / TN, co = row - ab * TN;
                val = *(const uint4*)(w + ((int64_t)ab * cout_p + co0 + co) * cin_p + k0 + part * VE);
            }
            rw[i] = val;
        }
    };
    auto lstore = [&]() {
#pragma unroll
        for (int i = 0; i < NXV; ++i) {
            const int v = threadIdx.x + i * CT;
            if (v < nxv) {
                const int px = v / vpp, part = v - px * vpp;
                *(uint4*)&xin[px * PS + part * VE] = rx[i];
            }
        }
#pragma unroll
        for (int i = 0; i < NWV; ++i) {
            const int v = threadIdx.x + i * CT;
            if (v < nwv) {
                const int row = v / vpp, part = v - row * vpp;
                *(uint4*)&wl[row * PS + part * VE] = rw[i];
            }
        }
    };
    gload(0);
    asm volatile("" ::: "memory");
    if (skipped) return;   // uniform over the block
    for (int k0 = 0; k0 < cin_p; k0 += ks) {
        __syncthreads();
        lstore();
        __syncthreads();
        if (k0 + ks < cin_p) gload(k0 + ks);
        const T* xb = &xin[(wv * 16 + lr) * PS + lg * P::GW];
        const T* wb = &wl[lr * PS + lg * P::GW];
        if (ks % (4 * P::GW) == 0) {   // whole steps: unrolled, stops after ks channels
#pragma unroll
            for (int st = 0; st < KSM / P::GW / 4; ++st) {
                if (4 * st * P::GW >= ks) break;
                const Frag b = P::load(xb + 4 * st * P::GW);
#pragma unroll
                for (int ab = 0; ab < 4; ++ab)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb)
                        acc[ab][cb] = P::mma(P::load(wb + (ab * TN + cb * 16) * PS + 4 * st * P::GW), b, acc[ab][cb]);
            }
        } else {
            const int groups = ks / P::GW;
            for (int st = 0; st < (groups + 3) / 4; ++st) {
                const int cg = 4 * st + lg;
                const Frag b = cg < groups ? P::load(xb + 4 * st * P::GW) : P::zero();
#pragma unroll
                for (int ab = 0; ab < 4; ++ab)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        const Frag a = cg < groups ? P::load(wb + (ab * TN + cb * 16) * PS + 4 * st * P::GW) : P::zero();
                        acc[ab][cb] = P::mma(a, b, acc[ab][cb]);
                    }
            }
        }
    }
    const int gx = ix0 + wv * 16 + lr;
    if (gx >= W) return;
    T* ys = y + (int64_t)bz * plane * 4 * cout_p;
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) {
        const int oy = 2 * iy + (ab >> 1), ox = 2 * gx + (ab & 1);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int co = co0 + cb * 16;
            T* dst = ys + ((int64_t)oy * (2 * W) + ox) * cout_p + co;
            Acc t[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) t[r] = acc[ab][cb][r] + bias[co + P::row_of(lg, r)];
            store_rows<P>(dst + P::row_of(lg, 0), t);
        }
    }
}

template <class P, int TN>
__global__ __launch_bounds__(CT) void k_convT2(const typename P::T* __restrict__ x, int cin_p,
                                               const typename P::T* __restrict__ w,
                                               const typename P::Acc* __restrict__ bias,
                                               typename P::T* __restrict__ y, int cout_p, int H, int W, int ck,
                                               const int* __restrict__ skip) {
    const int ncb_tot = cout_p / TN;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    int v = xcd_linear(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nblk);
    const int cbi = v % ncb_tot;
    v /= ncb_tot;
    const int txi = v % gridDim.x;
    v /= gridDim.x;
    const int tyi = v % gridDim.y;
    const int bz = v / gridDim.y;
    convT2_tile<P, TN>(x, cin_p, w, bias, y, cout_p, H, W, ck, bz, cbi * TN, tyi, txi * 64, skip);
}

template <class P, int TN>
__global__ __launch_bounds__(CT) void k_convT2_jobs(const TileJob* __restrict__ jobs, const LayerIO* __restrict__ io,
                                                    const typename P::T* __restrict__ w,
                                                    const typename P::Acc* __restrict__ bias, int cin_p, int cout_p,
                                                    int ck) {
    const TileJob jb = jobs[xcd_linear(blockIdx.x, gridDim.x)];
    const LayerIO d = io[jb.sys];
    if (d.stop && *d.stop) return;
    convT2_tile<P, TN>((const typename P::T*)d.x0, cin_p, w, bias, (typename P::T*)d.y, cout_p, d.H, d.W, ck, 0, jb.c0,
                       jb.ty0, jb.tx0);
}

// Transposed convolution with every input channel in one stage (cin_p a multiple of 4 GW, at
// most 4 CK), weight-stationary: a block keeps the weights of its TN output channels in LDS and
// runs the 64-pixel input row segments [t_beg, t_end) of one sample (segment t: input row
// t / nseg, columns 64 (t % nseg) ..; xs and ys at the sample). As in conv3_ws_body, wavefronts
// 4-7 only load (K register sets, one segment per step into a double-buffered LDS patch) and
// wavefronts 0-3 only run the matrix cores and store, one barrier per step; the MFMA steps and
// the epilogue are convT2_tile's (the same result bits).
template <class P, int TN, int K>
__device__ __forceinline__ void convT2_ws_body(const typename P::T* __restrict__ xs, typename P::T* __restrict__ ys,
                                               const typename P::T* __restrict__ w,
                                               const typename P::Acc* __restrict__ bias, int cin_p, int cout_p,
                                               int W, int co0, int t_beg, int t_end) {
    using T = typename P::T;
    using Acc = typename P::Acc;
    using AccV = typename P::AccV;
    using Frag = typename P::Frag;
    constexpr int KSM = convT2_ksmax<P>();
    constexpr int PS = KSM + 16 / (int)sizeof(T);
    constexpr int VE = 16 / sizeof(T);
    constexpr int NCB = TN / 16;
    constexpr int NXA = (64 * KSM / VE + CT - 1) / CT;                    // per loader thread
    constexpr int NWV = (4 * TN * KSM / VE + WS_THREADS - 1) / WS_THREADS;   // per thread
    __shared__ __attribute__((aligned(16))) T xin[2 * 64 * PS];
    __shared__ __attribute__((aligned(16))) T wl[4 * TN * PS];
    const int nseg = (W + 63) / 64;
    const int vpp = cin_p / VE;
    const int nxv = 64 * vpp, nwv = 4 * TN * vpp;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool loader = wv >= 4;
    const int lt = threadIdx.x - CT;
    const int lr = lane & 15, lg = lane >> 4;
    {   // the block's weights (every wavefront): [4 parities][TN][cin_p] into LDS rows
        uint4 rw[NWV];
#pragma unroll
        for (int i = 0; i < NWV; ++i) {
            const int v = threadIdx.x + i * WS_THREADS;
            rw[i] = uint4{0, 0, 0, 0};
            if (v < nwv) {
                const int row = v / vpp, part = v - row * vpp;
                const int ab = row / TN, co = row - ab * TN;
                rw[i] = *(const uint4*)(w + ((int64_t)ab * cout_p + co0 + co) * cin_p + part * VE);
            }
        }
#pragma unroll
        for (int i = 0; i < NWV; ++i) {
            const int v = threadIdx.x + i * WS_THREADS;
            if (v < nwv) {
                const int row = v / vpp, part = v - row * vpp;
                *(uint4*)&wl[row * PS + part * VE] = rw[i];
            }
        }
    }
    // loader: segment t into ra_, every lane loading (from pixel 0 of the row where its pixel is
    // past the row's end; ok_ marks the others), so that the loads in flight do not depend on data
    auto gload = [&](int t, uint4 (&ra_)[NXA], uint32_t& ok_) {
        const int iy = t / nseg, ix0 = (t - iy * nseg) * 64;
        ok_ = 0;
#pragma unroll
        for (int i = 0; i < NXA; ++i) {
            const int vv = min(lt + i * CT, nxv - 1);
            const int px = vv / vpp, part = vv - px * vpp;
            const int gx = ix0 + px;
            const bool in = gx < W;
            ok_ |= (in ? 1u : 0u) << i;
            ra_[i] = *(const uint4*)(xs + ((int64_t)iy * W + (in ? gx : 0)) * cin_p + part * VE);
        }
    };
    auto lstore = [&](int b, const uint4 (&ra_)[NXA], uint32_t ok_) {
#pragma unroll
        for (int i = 0; i < NXA; ++i) {
            const int vv = lt + i * CT;
            if (vv < nxv) {
                const int px = vv / vpp, part = vv - px * vpp;
                *(uint4*)&xin[b * 64 * PS + px * PS + part * VE] = ((ok_ >> i) & 1u) ? ra_[i] : uint4{0, 0, 0, 0};
            }
        }
    };
    uint4 ra[K][NXA];
    uint32_t ok[K];
    if (loader) {
#pragma unroll
        for (int u = 0; u < K; ++u) gload(min(t_beg + u, t_end - 1), ra[u], ok[u]);
        lstore(0, ra[0], ok[0]);
    }
    __syncthreads();
    Acc bpre[NCB][4];
    auto compute = [&](int t, int b) {
        AccV acc[4][NCB];
#pragma unroll
        for (int ab = 0; ab < 4; ++ab)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[ab][cb][r] = 0;
        const T* xb = &xin[b * 64 * PS + (wv * 16 + lr) * PS + lg * P::GW];
        const T* wb = &wl[lr * PS + lg * P::GW];
#pragma unroll
        for (int st = 0; st < KSM / P::GW / 4; ++st) {
            if (4 * st * P::GW >= cin_p) break;
            const Frag bx = P::load(xb + 4 * st * P::GW);
#pragma unroll
            for (int ab = 0; ab < 4; ++ab)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                    acc[ab][cb] = P::mma(P::load(wb + (ab * TN + cb * 16) * PS + 4 * st * P::GW), bx, acc[ab][cb]);
        }
        const int iy = t / nseg, ix0 = (t - iy * nseg) * 64;
        const int gx = ix0 + wv * 16 + lr;
        if (gx >= W) return;
#pragma unroll
        for (int ab = 0; ab < 4; ++ab) {
            const int oy = 2 * iy + (ab >> 1), ox = 2 * gx + (ab & 1);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                T* dst = ys + ((int64_t)oy * (2 * W) + ox) * cout_p + co0 + cb * 16;
                Acc tv[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) tv[r] = acc[ab][cb][r] + bpre[cb][r];
                store_rows<P>(dst + P::row_of(lg, 0), tv);
            }
        }
    };
    // the two roles run separate loops with one barrier per step (as conv3_ws_body)
    if (loader) {
        for (int t0 = t_beg; t0 < t_end; t0 += K) {
#pragma unroll
            for (int u = 0; u < K; ++u) {
                const int t = t0 + u;
                if (t < t_end) {
                    const int b = (t - t_beg) & 1;
                    if (t + 1 < t_end) lstore(b ^ 1, ra[(u + 1) % K], ok[(u + 1) % K]);
                    gload(min(t + K, t_end - 1), ra[u], ok[u]);
                    __syncthreads();
                }
            }
        }
    } else {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) bpre[cb][r] = bias[co0 + cb * 16 + P::row_of(lg, r)];
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the bias is in registers before the loop
        for (int t = t_beg; t < t_end; ++t) {
            compute(t, (t - t_beg) & 1);
            __syncthreads();
        }
    }
}

// Ragged batch: job = (system, first output channel, t_beg, t_end) in (sys, c0, ty0, tx0).
template <class P, int TN, int K>
__global__ __launch_bounds__(WS_THREADS) void k_convT2_ws_jobs(const TileJob* __restrict__ jobs,
                                                               const LayerIO* __restrict__ io,
                                                               const typename P::T* __restrict__ w,
                                                               const typename P::Acc* __restrict__ bias, int cin_p,
                                                               int cout_p) {
    const TileJob jb = jobs[xcd_linear(blockIdx.x, gridDim.x)];
    const LayerIO d = io[jb.sys];
    if (d.stop && *d.stop) return;
    convT2_ws_body<P, TN, K>((const typename P::T*)d.x0, (typename P::T*)d.y, w, bias, cin_p, cout_p, d.W, jb.c0,
                             jb.ty0, jb.tx0);
}

// grid: x = segment groups (tpb segments each), y = channel blocks, z = samples; logical block
// order: channel block fastest, then segment group, then sample.
template <class P, int TN, int K>
__global__ __launch_bounds__(WS_THREADS) void k_convT2_ws(const typename P::T* __restrict__ x, int cin_p,
                                                          const typename P::T* __restrict__ w,
                                                          const typename P::Acc* __restrict__ bias,
                                                          typename P::T* __restrict__ y, int cout_p, int H, int W,
                                                          int tpb, const int* __restrict__ skip) {
    if (skip && *skip) return;   // uniform over the grid
    const int ncb_tot = gridDim.y;
    const int ngrp = gridDim.x;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    int v = xcd_linear(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nblk);
    const int cbi = v % ncb_tot;
    v /= ncb_tot;
    const int grp = v % ngrp;
    const int bz = v / ngrp;
    const int nt = H * ((W + 63) / 64);
    const int t_beg = grp * tpb, t_end = min(nt, t_beg + tpb);
    const int64_t plane = (int64_t)H * W;
    convT2_ws_body<P, TN, K>(x + (int64_t)bz * plane * cin_p, y + (int64_t)bz * plane * 4 * cout_p, w, bias, cin_p,
                             cout_p, W, cbi * TN, t_beg, t_end);
}

static int pick_tn(int cout_p) { return cout_p % 64 == 0 ? 64 : (cout_p % 32 == 0 ? 32 : 16); }

int conv3_batch_tn(int cout_p, int64_t tiles) {
    int tn = cout_p % 64 == 0 ? 64 : (cout_p % 32 == 0 ? 32 : 16);
    while (tn > 16 && tiles * (cout_p / tn) < 512) tn /= 2;
    return tn;
}
// 16-channel blocks (every padded channel count is a multiple of 16): the kernel runs one tile per
// block with one load stage, and the 16-channel form's registers and LDS let 4 blocks share a CU
// instead of 2, hiding more of each block's load latency (faster on the serving mix, where the
// transposed layers are bound by that latency rather than by the bytes they move)
int convT2_batch_tn(int /*cout_p*/) {
    return 16;
}

template <class P>
static int convT2_stage(int cin_p) {
    int ks = convT2_ksmax<P>();
    while (ks > 1 && cin_p % ks) ks /= 2;
    return ks;
}

template <class P>
static int chunk_for(int cin_p, int c0, int c1) {
    int ck = P::CK;
    if (cin_p < ck) ck = cin_p;
    if (c1 > 0) {
        if (c0 < ck) ck = c0;
        if (c1 < ck) ck = c1;
    }
    return ck;
}

template <class P>
int launch_conv3(const typename P::T* x0, int c0, const typename P::T* x1, int c1, const typename P::T* w,
                 const typename P::Acc* bias, typename P::T* y, int cout_p, typename P::T* ypool, int H, int W,
                 int batch, bool relu, const int* skip, hipStream_t s, Conv3Out ex, ConvCfg cfg,
                 typename P::Acc* splitbuf) {
    const int cin_p = c0 + c1;
    const int ck = chunk_for<P>(cin_p, c0, c1);
    constexpr int VE = 16 / sizeof(typename P::T);
    if (cout_p % 16 || cin_p % ck || c0 % ck || ck % VE || ck % P::GW || (ypool && (H % 2 || W % 2))) {
        set_error("conv3: unsupported channel / size combination");
        return HZ_ERR_ARG;
    }
    const int rpw = cfg.rpw == 4 ? 4 : 2;
    if (cfg.tpb > 1 && !ex.head_w && !ex.split && !ex.mask0_ && !ex.mask1_ && bias &&
        conv3_ws_ok<P>(cfg.tn, rpw, c0, c1, cout_p)) {
        // weight-stationary form: all weights of the block's channels in LDS, cfg.tpb tiles per block
        const int tn = cfg.tn, th = 4 * rpw;
        const int ntiles = ((W + TW - 1) / TW) * ((H + th - 1) / th);
        const int ngrp = (ntiles + cfg.tpb - 1) / cfg.tpb;
        const int nch = cin_p / P::CK;
        dim3 grid(ngrp, cout_p / tn, batch);
        if (conv3_ws_small<P>(c0, c1)) {
            if (ypool) {
                set_error("conv3: the weight-stationary form of a one-k-group input has no pooled output");
                return HZ_ERR_ARG;
            }
            if constexpr (std::is_same<P, PolBF16>::value) {
#define HZ_WS8(TNV, R, KV)                                                                                     \
    hipLaunchKernelGGL((k_conv3_ws8<P, TNV, R, KV>), grid, dim3(WS_THREADS), 0, s, x0, c0, w, bias, y, cout_p, H, W, \
                       relu ? 1 : 0, cfg.tpb, skip)
#define HZ_WS8K(TNV, R)                                     \
    if constexpr (R == 2) {                                 \
        if (cfg.ns >= 4) { HZ_WS8(TNV, R, 4); }             \
        else if (cfg.ns == 3) { HZ_WS8(TNV, R, 3); }        \
        else { HZ_WS8(TNV, R, 2); }                         \
    } else {                                                \
        HZ_WS8(TNV, R, 2);                                  \
    }
#define HZ_WS8T(R)                             \
    if (tn == 64) { HZ_WS8K(64, R) }           \
    else if (tn == 32) { HZ_WS8K(32, R) }      \
    else { HZ_WS8K(16, R) }
                if (rpw == 4) { HZ_WS8T(4) } else { HZ_WS8T(2) }
#undef HZ_WS8T
#undef HZ_WS8K
#undef HZ_WS8
            }
            HZ_LAUNCH_CHECK();
            return HZ_OK;
        }
#define HZ_WS1(TNV, PL, R, WC, KV)                                                                           \
    hipLaunchKernelGGL((k_conv3_ws<P, TNV, PL, R, WC, KV>), grid, dim3(WS_THREADS), 0, s, x0, c0, x1, c1, w, bias, \
                       y, cout_p, ypool, H, W, relu ? 1 : 0, cfg.tpb, skip)
#define HZ_WS(TNV, PL, R, WC)                                             \
    if constexpr (R == 2) {                                               \
        if (cfg.ns >= 4 && WC <= 2) { HZ_WS1(TNV, PL, R, WC, 4); }        \
        else if (cfg.ns == 3) { HZ_WS1(TNV, PL, R, WC, 3); }              \
        else { HZ_WS1(TNV, PL, R, WC, 2); }                               \
    } else {                                                              \
        HZ_WS1(TNV, PL, R, WC, 2);                                        \
    }
#define HZ_WSW(TNV, PL, R)                                                                        \
    if (nch == 1) {                                                                                \
        if constexpr (conv3_ws_lds<P>(TNV, R, 1) <= 160 * 1024) { HZ_WS(TNV, PL, R, 1); }          \
    } else if (nch == 2) {                                                                         \
        if constexpr (conv3_ws_lds<P>(TNV, R, 2) <= 160 * 1024) { HZ_WS(TNV, PL, R, 2); }          \
    } else if constexpr (conv3_ws_lds<P>(TNV, R, 4) <= 160 * 1024) { HZ_WS(TNV, PL, R, 4); }
#define HZ_WST(PL, R)                        \
    if (tn == 64) { HZ_WSW(64, PL, R) }      \
    else if (tn == 32) { HZ_WSW(32, PL, R) } \
    else { HZ_WSW(16, PL, R) }
        if constexpr (std::is_same<P, PolBF16>::value) {
            if (ypool) {
                if (rpw == 4) { HZ_WST(true, 4) } else { HZ_WST(true, 2) }
            } else {
                if (rpw == 4) { HZ_WST(false, 4) } else { HZ_WST(false, 2) }
            }
        }
#undef HZ_WST
#undef HZ_WSW
#undef HZ_WS
#undef HZ_WS1
        HZ_LAUNCH_CHECK();
        return HZ_OK;
    }
    int ksplit = cfg.ksplit < 1 ? 1 : cfg.ksplit;
    if (ksplit > cin_p / ck) ksplit = cin_p / ck;
    if (ksplit > 1 && (!splitbuf || ex.split || ex.mask0_ || ex.mask1_)) ksplit = 1;
    const int th = 4 * rpw;
    int tn = cfg.tn;
    if (tn != 16 && tn != 32 && tn != 64) {
        // widest channel tile that still gives the GPU enough blocks (256 CUs)
        tn = pick_tn(cout_p);
        const int64_t tiles = (int64_t)((W + TW - 1) / TW) * ((H + th - 1) / th) * batch;
        while (tn > 16 && tiles * (cout_p / tn) < 512) tn /= 2;
    }
    while (cout_p % tn) tn /= 2;
    if (ex.head_w) {
        if ((cout_p != 16 && cout_p != 32 && cout_p != 64) || ypool || ex.split || batch != 1 || !ex.head_z ||
            (!ex.head_sc && !(ex.head_fixed_s > 0))) {
            set_error("conv3: fused head needs 16, 32 or 64 channels, one sample and no pooling");
            return HZ_ERR_ARG;
        }
        tn = cout_p;
        ksplit = 1;
    }
    if (ex.split > 0) {
        if (ex.split % 16 || ex.split >= cout_p || (ypool && ex.split)) {
            set_error("conv3: bad output split");
            return HZ_ERR_ARG;
        }
        while (ex.split % tn || (cout_p - ex.split) % tn) tn /= 2;
    }
    dim3 grid((W + TW - 1) / TW, (H + th - 1) / th, (cout_p / tn) * batch * ksplit);
    const int64_t sstride = (int64_t)batch * H * W * cout_p;
    typename P::Acc* sp = ksplit > 1 ? splitbuf : nullptr;
    const bool kpool = ypool && ksplit == 1;
    // chunks per LDS stage: BF16 only, where the stage fits in LDS (conv3_stages_ok)
    int ns = cfg.ns;
    if (!conv3_stages_ok<P>(tn, rpw, ns) || ex.head_w) ns = 1;
#define HZ_C3(TNV, PL, R, NSV)                                                                                  \
    hipLaunchKernelGGL((k_conv3<P, TNV, PL, R, NSV>), grid, dim3(CT), 0, s, x0, c0, x1, c1, w, bias, y, cout_p, \
                       kpool ? ypool : nullptr, H, W, relu ? 1 : 0, ck, skip, ex, ksplit, sp, sstride)
#define HZ_C3N(TNV, PL, R)                                                    \
    if constexpr (std::is_same<P, PolBF16>::value) {                          \
        if (ns == 2) HZ_C3(TNV, PL, R, 2);                                    \
        else if (ns == 4) {                                                   \
            if constexpr (conv3_stages_ok<P>(TNV, R, 4)) HZ_C3(TNV, PL, R, 4); \
        } else HZ_C3(TNV, PL, R, 1);                                          \
    } else {                                                                  \
        HZ_C3(TNV, PL, R, 1);                                                 \
    }
#define HZ_C3T(PL, R)                       \
    if (tn == 64) { HZ_C3N(64, PL, R) }     \
    else if (tn == 32) { HZ_C3N(32, PL, R) } \
    else { HZ_C3N(16, PL, R) }
    if (kpool) {
        if (rpw == 4) { HZ_C3T(true, 4) } else { HZ_C3T(true, 2) }
    } else {
        if (rpw == 4) { HZ_C3T(false, 4) } else { HZ_C3T(false, 2) }
    }
#undef HZ_C3T
#undef HZ_C3N
#undef HZ_C3
    HZ_LAUNCH_CHECK();
    if (ksplit > 1) {
        const int64_t items = ypool ? (int64_t)batch * (H / 2) * (W / 2) * cout_p : (int64_t)batch * H * W * cout_p;
        const unsigned g = (unsigned)((items + 255) / 256);
        if (ypool)
            hipLaunchKernelGGL((k_splitk_epilogue<P, true>), dim3(g), dim3(256), 0, s, splitbuf, ksplit, sstride, bias,
                               y, ypool, H, W, cout_p, batch, relu ? 1 : 0, skip);
        else
            hipLaunchKernelGGL((k_splitk_epilogue<P, false>), dim3(g), dim3(256), 0, s, splitbuf, ksplit, sstride,
                               bias, y, ypool, H, W, cout_p, batch, relu ? 1 : 0, skip);
        HZ_LAUNCH_CHECK();
    }
    return HZ_OK;
}

template <class P>
bool conv3_up_ok(int c0, int c1, int cd, int H, int W) {
    if constexpr (!std::is_same<P, PolBF16>::value) {
        return false;
    } else {
        return c0 > 0 && c1 > 0 && c0 % P::CK == 0 && c1 % P::CK == 0 && cd > 0 && cd <= UP_CDMAX &&
               cd % (4 * P::GW) == 0 && H % 2 == 0 && W % 2 == 0;
    }
}

template <class P>
int launch_conv3_up(const typename P::T* x0, int c0, UpIn up, int c1, const typename P::T* w,
                    const typename P::Acc* bias, typename P::T* y, int cout_p, int H, int W, int batch,
                    const int* skip, hipStream_t s, ConvCfg cfg) {
    if (!conv3_up_ok<P>(c0, c1, up.cd, H, W) || cout_p % 16 || !up.d || !up.wt || !up.bt) {
        set_error("conv3_up: unsupported channel / size combination");
        return HZ_ERR_ARG;
    }
    if constexpr (std::is_same<P, PolBF16>::value) {
        const int rpw = cfg.rpw == 4 ? 4 : 2;
        const int th = 4 * rpw;
        int tn = cfg.tn;
        if (tn != 16 && tn != 32 && tn != 64) {
            tn = pick_tn(cout_p);
            const int64_t tiles = (int64_t)((W + TW - 1) / TW) * ((H + th - 1) / th) * batch;
            while (tn > 16 && tiles * (cout_p / tn) < 512) tn /= 2;
        }
        while (cout_p % tn) tn /= 2;
        dim3 grid((W + TW - 1) / TW, (H + th - 1) / th, (cout_p / tn) * batch);
        // LDS and fragment registers sized for the coarse channel count (64 or 128)
#define HZ_CU(TNV, R)                                                                                             \
    if (up.cd <= 64)                                                                                             \
        hipLaunchKernelGGL((k_conv3_up<P, TNV, R, 64>), grid, dim3(CT), 0, s, x0, c0, up, c1, w, bias, y, cout_p, \
                           H, W, skip);                                                                          \
    else                                                                                                         \
        hipLaunchKernelGGL((k_conv3_up<P, TNV, R, UP_CDMAX>), grid, dim3(CT), 0, s, x0, c0, up, c1, w, bias, y,    \
                           cout_p, H, W, skip)
        if (rpw == 4) {
            if (tn == 64) HZ_CU(64, 4);
            else if (tn == 32) HZ_CU(32, 4);
            else HZ_CU(16, 4);
        } else {
            if (tn == 64) HZ_CU(64, 2);
            else if (tn == 32) HZ_CU(32, 2);
            else HZ_CU(16, 2);
        }
#undef HZ_CU
        HZ_LAUNCH_CHECK();
    }
    return HZ_OK;
}

template <class P>
int launch_convT2(const typename P::T* x, int cin_p, const typename P::T* w, const typename P::Acc* bias,
                  typename P::T* y, int cout_p, int H, int W, int batch, const int* skip, hipStream_t s) {
    const int ck = convT2_stage<P>(cin_p);
    constexpr int VE = 16 / sizeof(typename P::T);
    if (cout_p % 16 || ck < VE || cin_p % ck || ck % VE) {
        set_error("convT2: unsupported channel combination");
        return HZ_ERR_ARG;
    }
    if constexpr (std::is_same<P, PolBF16>::value) {
        // the weight-stationary form (16-channel blocks, 4-32 row segments per block) where the input
        // channels fit one stage and it gives at least 256 blocks (the same result bits)
        if (convT2_ws_ok<P>(cin_p, cout_p, 16)) {
            const int nt = H * ((W + 63) / 64);
            const int64_t ncb = cout_p / 16;
            int tpb = 32;
            while (tpb > 4 && (int64_t)((nt + tpb - 1) / tpb) * ncb * batch < 1024) tpb /= 2;
            if ((int64_t)((nt + tpb - 1) / tpb) * ncb * batch >= 256) {
                dim3 g((nt + tpb - 1) / tpb, (unsigned)ncb, batch);
                hipLaunchKernelGGL((k_convT2_ws<P, 16, 2>), g, dim3(WS_THREADS), 0, s, x, cin_p, w, bias, y, cout_p, H,
                                   W, tpb, skip);
                HZ_LAUNCH_CHECK();
                return HZ_OK;
            }
        }
    }
    const int tn = cout_p % 32 == 0 ? 32 : 16;
    dim3 grid((W + 63) / 64, H, (cout_p / tn) * batch);
    if (tn == 32)
        hipLaunchKernelGGL((k_convT2<P, 32>), grid, dim3(CT), 0, s, x, cin_p, w, bias, y, cout_p, H, W, ck, skip);
    else
        hipLaunchKernelGGL((k_convT2<P, 16>), grid, dim3(CT), 0, s, x, cin_p, w, bias, y, cout_p, H, W, ck, skip);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

template <class P>
int conv_chunk(int cin_p, int c0, int c1) { return chunk_for<P>(cin_p, c0, c1); }

template <class P>
int launch_conv3_jobs(const TileJob* jobs, int njobs, const LayerIO* io, const typename P::T* w,
                      const typename P::Acc* bias, int c0, int c1, int cout_p, int tn, int rpw, bool pool,
                      hipStream_t s) {
    if (njobs <= 0) return HZ_OK;
    const int ck = chunk_for<P>(c0 + c1, c0, c1);
#define HZ_C3J(TNV, PL, R)                                                                                         \
    hipLaunchKernelGGL((k_conv3_jobs<P, TNV, PL, R>), dim3(njobs), dim3(CT), 0, s, jobs, io, w, bias, c0, c1, cout_p, \
                       1, ck)
    if (rpw == 4) {
        if constexpr (std::is_same<P, PolBF16>::value) {
            if (tn != 32) {
                set_error("conv3 jobs: 16-row tiles use 32-channel blocks");
                return HZ_ERR_ARG;
            }
            if (pool) HZ_C3J(32, true, 4);
            else HZ_C3J(32, false, 4);
        } else {
            set_error("conv3 jobs: 16-row tiles are BF16 only");
            return HZ_ERR_ARG;
        }
    } else if (pool) {
        if (tn == 64) HZ_C3J(64, true, 2);
        else if (tn == 32) HZ_C3J(32, true, 2);
        else HZ_C3J(16, true, 2);
    } else {
        if (tn == 64) HZ_C3J(64, false, 2);
        else if (tn == 32) HZ_C3J(32, false, 2);
        else HZ_C3J(16, false, 2);
    }
#undef HZ_C3J
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

template <class P>
int launch_conv3_jobs_head(const TileJob* jobs, int njobs, const LayerIO* io, const typename P::T* w,
                           const typename P::Acc* bias, int c0, int c1, int cout_p, const typename P::T* head_w,
                           const typename P::Acc* head_b, int col, bool c128, hipStream_t s) {
    if (njobs <= 0) return HZ_OK;
    const int ck = chunk_for<P>(c0 + c1, c0, c1);
#define HZ_C3H(TNV)                                                                                      \
    hipLaunchKernelGGL((k_conv3_jobs_head<P, TNV>), dim3(njobs), dim3(CT), 0, s, jobs, io, w, bias, c0, c1, ck, \
                       head_w, head_b, col, c128 ? 1 : 0)
    if (cout_p == 64) HZ_C3H(64);
    else if (cout_p == 32) HZ_C3H(32);
    else if (cout_p == 16) HZ_C3H(16);
    else {
        set_error("conv3 jobs: fused head needs 16, 32 or 64 channels");
        return HZ_ERR_ARG;
    }
#undef HZ_C3H
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

template <class P>
int launch_conv3_ws_jobs(const TileJob* jobs, int njobs, const LayerIO* io, const typename P::T* w,
                         const typename P::Acc* bias, int c0, int c1, int cout_p, bool pool,
                         const typename P::T* head_w, const typename P::Acc* head_b, int col, bool c128,
                         hipStream_t s) {
    if (njobs <= 0) return HZ_OK;
    if constexpr (std::is_same<P, PolBF16>::value) {
        const int nch = (c0 + c1) / P::CK;
        if (!ws_jobs_ok<P>(c0, c1, cout_p) || (head_w && (pool || cout_p != WSJ_TN))) {
            set_error("conv3 jobs: the weight-stationary form needs BF16, 32-channel blocks, 1 or 2 input chunks");
            return HZ_ERR_ARG;
        }
#define HZ_WSJ(PL, WC, HD, SM)                                                                                  \
    hipLaunchKernelGGL((k_conv3_ws_jobs<P, WSJ_TN, PL, WSJ_RPW, WC, 2, HD, SM>), dim3(njobs), dim3(WS_THREADS), 0, \
                       s, jobs, io, w, bias, c0, c1, cout_p, head_w, head_b, col, c128 ? 1 : 0)
        if (conv3_ws_small<P>(c0, c1)) {
            if (head_w || pool) {
                set_error("conv3 jobs: an input of one k-group per tap has no fused head or pooling here");
                return HZ_ERR_ARG;
            }
            HZ_WSJ(false, 1, false, true);
        } else if (head_w) {
            if (nch == 1) HZ_WSJ(false, 1, true, false);
            else HZ_WSJ(false, 2, true, false);
        } else if (pool) {
            if (nch == 1) HZ_WSJ(true, 1, false, false);
            else HZ_WSJ(true, 2, false, false);
        } else {
            if (nch == 1) HZ_WSJ(false, 1, false, false);
            else HZ_WSJ(false, 2, false, false);
        }
#undef HZ_WSJ
        HZ_LAUNCH_CHECK();
        return HZ_OK;
    } else {
        set_error("conv3 jobs: the weight-stationary form is BF16 only");
        return HZ_ERR_ARG;
    }
}

template <class P>
int launch_convT2_ws_jobs(const TileJob* jobs, int njobs, const LayerIO* io, const typename P::T* w,
                          const typename P::Acc* bias, int cin_p, int cout_p, int tn, hipStream_t s) {
    if (njobs <= 0) return HZ_OK;
    if constexpr (std::is_same<P, PolBF16>::value) {
        if (!convT2_ws_ok<P>(cin_p, cout_p, tn)) {
            set_error("convT2 jobs: the weight-stationary form needs BF16 and one stage of input channels");
            return HZ_ERR_ARG;
        }
        if (tn == 32)
            hipLaunchKernelGGL((k_convT2_ws_jobs<P, 32, 2>), dim3(njobs), dim3(WS_THREADS), 0, s, jobs, io, w, bias,
                               cin_p, cout_p);
        else
            hipLaunchKernelGGL((k_convT2_ws_jobs<P, 16, 2>), dim3(njobs), dim3(WS_THREADS), 0, s, jobs, io, w, bias,
                               cin_p, cout_p);
        HZ_LAUNCH_CHECK();
        return HZ_OK;
    } else {
        set_error("convT2 jobs: the weight-stationary form is BF16 only");
        return HZ_ERR_ARG;
    }
}

template <class P>
int launch_conv3_ws_dgrad(const typename P::T* x0, int c0, const typename P::T* w, typename P::T* y0, int cout_p,
                          int H, int W, int batch, int split, typename P::T* y1, const typename P::T* mask0,
                          const typename P::T* mask1, hipStream_t s) {
    if constexpr (std::is_same<P, PolBF16>::value) {
        if (!conv3_ws_dgrad_ok<P>(c0, cout_p, split)) {
            set_error("conv3: the weight-stationary data gradient needs BF16, 1 or 2 input chunks and 32-channel parts");
            return HZ_ERR_ARG;
        }
        const int ntiles = ((W + TW - 1) / TW) * ((H + 15) / 16);
        const int ncb = cout_p / WSJ_TN;
        int tpb = 32;
        while (tpb > 4 && (int64_t)((ntiles + tpb - 1) / tpb) * ncb * batch < 1024) tpb /= 2;
        dim3 grid((ntiles + tpb - 1) / tpb, ncb, batch);
        if (c0 == P::CK)
            hipLaunchKernelGGL((k_conv3_ws_dgrad<P, WSJ_TN, WSJ_RPW, 1, 2>), grid, dim3(WS_THREADS), 0, s, x0, c0, w, y0,
                               cout_p, H, W, tpb, split, y1, mask0, mask1);
        else
            hipLaunchKernelGGL((k_conv3_ws_dgrad<P, WSJ_TN, WSJ_RPW, 2, 2>), grid, dim3(WS_THREADS), 0, s, x0, c0, w, y0,
                               cout_p, H, W, tpb, split, y1, mask0, mask1);
        HZ_LAUNCH_CHECK();
        return HZ_OK;
    } else {
        set_error("conv3: the weight-stationary data gradient is BF16 only");
        return HZ_ERR_ARG;
    }
}

template <class P>
int launch_convT2_jobs(const TileJob* jobs, int njobs, const LayerIO* io, const typename P::T* w,
                       const typename P::Acc* bias, int cin_p, int cout_p, int tn, hipStream_t s) {
    if (njobs <= 0) return HZ_OK;
    const int ck = convT2_stage<P>(cin_p);
    if (ck < 16 / (int)sizeof(typename P::T) || cin_p % ck) {
        set_error("convT2: unsupported channel combination");
        return HZ_ERR_ARG;
    }
    if (tn == 32)
        hipLaunchKernelGGL((k_convT2_jobs<P, 32>), dim3(njobs), dim3(CT), 0, s, jobs, io, w, bias, cin_p, cout_p, ck);
    else
        hipLaunchKernelGGL((k_convT2_jobs<P, 16>), dim3(njobs), dim3(CT), 0, s, jobs, io, w, bias, cin_p, cout_p, ck);
    HZ_LAUNCH_CHECK();
    return HZ_OK;
}

#define HZ_INST(P)                                                                                              \
    template int launch_conv3<P>(const P::T*, int, const P::T*, int, const P::T*, const P::Acc*, P::T*, int,     \
                                 P::T*, int, int, int, bool, const int*, hipStream_t, Conv3Out, ConvCfg,       \
                                 P::Acc*);                                                                     \
    template int launch_convT2<P>(const P::T*, int, const P::T*, const P::Acc*, P::T*, int, int, int, int,       \
                                  const int*, hipStream_t);                                                    \
    template int launch_conv3_jobs<P>(const TileJob*, int, const LayerIO*, const P::T*, const P::Acc*, int, int, \
                                      int, int, int, bool, hipStream_t);                                       \
    template int launch_conv3_jobs_head<P>(const TileJob*, int, const LayerIO*, const P::T*, const P::Acc*, int,   \
                                           int, int, const P::T*, const P::Acc*, int, bool, hipStream_t);       \
    template int launch_conv3_ws_jobs<P>(const TileJob*, int, const LayerIO*, const P::T*, const P::Acc*, int, int, \
                                         int, bool, const P::T*, const P::Acc*, int, bool, hipStream_t);        \
    template int launch_conv3_ws_dgrad<P>(const P::T*, int, const P::T*, P::T*, int, int, int, int, int, P::T*,   \
                                          const P::T*, const P::T*, hipStream_t);                               \
    template int launch_convT2_jobs<P>(const TileJob*, int, const LayerIO*, const P::T*, const P::Acc*, int, int, \
                                       int, hipStream_t);                                                      \
    template int launch_convT2_ws_jobs<P>(const TileJob*, int, const LayerIO*, const P::T*, const P::Acc*, int,    \
                                          int, int, hipStream_t);                                              \
    template int conv_chunk<P>(int, int, int);                                                                 \
    template bool conv3_up_ok<P>(int, int, int, int, int);                                                     \
    template int launch_conv3_up<P>(const P::T*, int, UpIn, int, const P::T*, const P::Acc*, P::T*, int, int, int, \
                                    int, const int*, hipStream_t, ConvCfg);
HZ_INST(PolBF16)
HZ_INST(PolF32)
HZ_INST(PolF64)
#undef HZ_INST

}  // namespace hz
