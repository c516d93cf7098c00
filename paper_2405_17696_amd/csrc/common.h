// Internal helpers of libhelm: complex arithmetic, vector loads, reductions,
// error reporting.  gfx950 only (64-wide wavefronts).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/helm.h"

namespace helm {

constexpr int WAVE = 64;

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);

#define HELM_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::helm::fail(HELM_EHIP, "%s:%d %s: %s", __FILE__, __LINE__, #call,    \
                                hipGetErrorString(e_));                                  \
    } while (0)

#define HELM_CHECK_LAUNCH() HELM_HIP(hipGetLastError())

// ---------------------------------------------------------------- kernel timer
// When a kernel name is armed, its launchers bracket each sampled launch (every
// launch, or every period-th one) with events on the launch stream and pass a
// device counter that the sampled launch's active blocks add their algorithmic
// work (bytes or flops) to.
struct KTimer {
    // true when this launch of the named kernel is sampled (timed and counted)
    bool armed(const char* name) const;
    // after every launch of the named kernel: advance the launch count and decide
    // whether the next launch is sampled (every period-th launch is)
    void next(const char* name, hipStream_t s);
    // at the start of each restart cycle of helm_solve: when whole cycles are
    // sampled, decide whether this one's launches are
    void step(hipStream_t s);
    unsigned long long* counter() const;
    bool capturing(hipStream_t s) const;
    void begin(hipStream_t s);
    void end(hipStream_t s);
    // Kept for the solver's replay loop; launches inside graphs are not timed.
    void replayed();
    void harvest();
    // Forget the event pairs of a previous graph (called before a new capture).
    void new_capture();
};
KTimer& ktimer();

#define TIMED_LAUNCH(name, stream, ...)                         \
    do {                                                        \
        const bool on_ = ::helm::ktimer().armed(name);          \
        if (on_) ::helm::ktimer().begin(stream);                \
        hipLaunchKernelGGL(__VA_ARGS__);                        \
        if (on_) ::helm::ktimer().end(stream);                  \
        ::helm::ktimer().next(name, stream);                    \
    } while (0)

// Launches recorded into a graph are neither timed nor counted.
#define WORK_COUNTER(name, stream) \
    (::helm::ktimer().armed(name) && !::helm::ktimer().capturing(stream) ? ::helm::ktimer().counter() : nullptr)

// The work counter is spread over WORK_SLOTS slots 128 bytes apart (block-index
// hashed), so that the one atomic per block does not serialise all blocks of a
// launch on a single address; helm_ktimer_read sums the slots.
constexpr int WORK_SLOTS = 64, WORK_SLOT_STRIDE = 16;
__device__ __forceinline__ void work_atomic(unsigned long long* c, unsigned long long v) {
    const unsigned slot = (blockIdx.x + 7u * blockIdx.y + 13u * blockIdx.z) % WORK_SLOTS;
    atomicAdd(c + slot * WORK_SLOT_STRIDE, v);
}
__device__ __forceinline__ void add_work(unsigned long long* c, unsigned long long v) {
    if (c && threadIdx.x == 0) work_atomic(c, v);
}

// ---------------------------------------------------------------- complex
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};
using c64 = cx<float>;
using c128 = cx<double>;

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) {
    cx<T> r;
    r.re = a;
    r.im = b;
    return r;
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk(s * a.re, s * a.im); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return mk(a.re, -a.im); }
template <typename T>
__host__ __device__ __forceinline__ T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cinv(cx<T> a) {
    T d = T(1) / (a.re * a.re + a.im * a.im);
    return mk(a.re * d, -a.im * d);
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cdot1(cx<T> a, cx<T> b) {
    return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <typename T, typename U>
__host__ __device__ __forceinline__ cx<T> ccast(cx<U> a) { return mk(T(a.re), T(a.im)); }

// ---------------------------------------------------------------- two-node loads
// Two consecutive nodes (16 B for c64, 32 B for c128), always 16-B aligned
// because node pairs start at even indices.
template <typename T>
struct pair2 {
    cx<T> a, b;
};
__device__ __forceinline__ pair2<float> ld_pair(const c64* p) {
    float4 v = *reinterpret_cast<const float4*>(p);
    return {mk(v.x, v.y), mk(v.z, v.w)};
}
__device__ __forceinline__ pair2<double> ld_pair(const c128* p) {
    double2 v0 = reinterpret_cast<const double2*>(p)[0];
    double2 v1 = reinterpret_cast<const double2*>(p)[1];
    return {mk(v0.x, v0.y), mk(v1.x, v1.y)};
}
__device__ __forceinline__ void st_pair(c64* p, pair2<float> v) {
    *reinterpret_cast<float4*>(p) = make_float4(v.a.re, v.a.im, v.b.re, v.b.im);
}
__device__ __forceinline__ void st_pair(c128* p, pair2<double> v) {
    reinterpret_cast<double2*>(p)[0] = make_double2(v.a.re, v.a.im);
    reinterpret_cast<double2*>(p)[1] = make_double2(v.b.re, v.b.im);
}

// ---------------------------------------------------------------- reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

}  // namespace helm
