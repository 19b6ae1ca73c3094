// Shared device/host helpers of the gfx950 library: complex arithmetic on
// float2/double2, BF16 conversion, wavefront reductions, error plumbing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <chrono>
#include <string>

#include "hz.h"

namespace hz {

// ----------------------------------------------------------------- errors

void set_error(const std::string& msg);
void clear_error();

#define HZ_CHECK_ARG(cond, msg)                 \
    do {                                        \
        if (!(cond)) {                          \
            ::hz::set_error(msg);               \
            return HZ_ERR_ARG;                  \
        }                                       \
    } while (0)

#define HZ_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            ::hz::set_error(std::string(#call) + ": " + hipGetErrorString(e_));               \
            return HZ_ERR_HIP;                                                                \
        }                                                                                     \
    } while (0)

#define HZ_LAUNCH_CHECK()                                                                     \
    do {                                                                                      \
        hipError_t e_ = hipGetLastError();                                                    \
        if (e_ != hipSuccess) {                                                               \
            ::hz::set_error(std::string("kernel launch: ") + hipGetErrorString(e_));          \
            return HZ_ERR_HIP;                                                                \
        }                                                                                     \
    } while (0)

#define HZ_TRY(call)                 \
    do {                             \
        int rc_ = (call);            \
        if (rc_ < 0) return rc_;     \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Process-wide identity of problem and network handles (never reused, unlike addresses).
uint64_t next_handle_uid();
// Drop the solver's kept graphs that refer to the handle with this identity (called when a
// problem or a network is destroyed; defined in fgmres.hip).
void fgmres_graph_cache_evict(uint64_t uid);

// Bump allocator over a caller workspace; every carve is 256-byte aligned.
struct Carver {
    char* base;
    size_t off = 0;
    size_t cap;
    Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
    template <typename T>
    T* take(size_t count) {
        off = align_up(off, 256);
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
    bool fits() const { return off <= cap; }
};

// ----------------------------------------------------------------- complex

template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };
template <typename T> using cplx_t = typename cplx<T>::type;

template <typename C> __host__ __device__ inline C cmul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <typename C> __host__ __device__ inline C cmulc(C a, C b) {
    return C{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename C> __host__ __device__ inline C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __host__ __device__ inline C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __host__ __device__ inline C cconj(C a) { return C{a.x, -a.y}; }
__host__ __device__ inline double2 to_d2(float2 a) { return double2{a.x, a.y}; }
__host__ __device__ inline double2 to_d2(double2 a) { return a; }
template <typename C> __host__ __device__ inline C from_d2(double2 a);
template <> __host__ __device__ inline float2 from_d2<float2>(double2 a) { return float2{(float)a.x, (float)a.y}; }
template <> __host__ __device__ inline double2 from_d2<double2>(double2 a) { return a; }

// ----------------------------------------------------------------- bf16

typedef uint16_t bf16_t;

// Round-to-nearest-even FP32 -> BF16, NaN preserving (quiet bit set).
__host__ __device__ inline bf16_t f2bf(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (bf16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(bf16_t b) { return __builtin_bit_cast(float, ((uint32_t)b) << 16); }

// ----------------------------------------------------------------- reductions

// Sum over the 64 lanes of a wavefront (every lane receives the result).
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// GPU time between two events on the solve's stream, summed per phase.
struct PhaseTimer {
    hipEvent_t ev[2] = {nullptr, nullptr};
    double ms[HZ_NPHASE] = {0, 0, 0, 0};
    int create() {
        for (auto& e : ev) HZ_HIP(hipEventCreate(&e));
        return HZ_OK;
    }
    // after a synchronisation of the stream: adds the time from ev[0] to ev[1]
    int add(int phase) {
        float t = 0.f;
        HZ_HIP(hipEventElapsedTime(&t, ev[0], ev[1]));
        ms[phase] += t;
        return HZ_OK;
    }
    ~PhaseTimer() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

}  // namespace hz
