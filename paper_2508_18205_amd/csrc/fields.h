// Field storage helpers: FP64, FP32 and BF16 storage with FP64/FP32 arithmetic.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct bf16s {
    uint16_t b;
};

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
// round to nearest even
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <typename TS> struct Store;

template <> struct Store<double> {
    using C = double;
    __device__ __forceinline__ static double ld1(const double* p, int64_t i) { return p[i]; }
    __device__ __forceinline__ static void st1(double* p, int64_t i, double v) { p[i] = v; }
    __device__ __forceinline__ static void ld2(const double* p, int64_t i, double& x, double& y) {
        const double2 v = reinterpret_cast<const double2*>(p)[i];
        x = v.x;
        y = v.y;
    }
    __device__ __forceinline__ static void st2(double* p, int64_t i, double x, double y) {
        reinterpret_cast<double2*>(p)[i] = make_double2(x, y);
    }
    __device__ __forceinline__ static void ld3(const double* p, int64_t i, double& x, double& y, double& z) {
        const double2 a = reinterpret_cast<const double2*>(p)[2 * i];
        const double b = p[4 * i + 2];
        x = a.x;
        y = a.y;
        z = b;
    }
    __device__ __forceinline__ static void st3(double* p, int64_t i, double x, double y, double z) {
        reinterpret_cast<double2*>(p)[2 * i] = make_double2(x, y);
        reinterpret_cast<double2*>(p)[2 * i + 1] = make_double2(z, 0.0);
    }
};

template <> struct Store<float> {
    using C = float;
    __device__ __forceinline__ static float ld1(const float* p, int64_t i) { return p[i]; }
    __device__ __forceinline__ static void st1(float* p, int64_t i, float v) { p[i] = v; }
    __device__ __forceinline__ static void ld2(const float* p, int64_t i, float& x, float& y) {
        const float2 v = reinterpret_cast<const float2*>(p)[i];
        x = v.x;
        y = v.y;
    }
    __device__ __forceinline__ static void st2(float* p, int64_t i, float x, float y) {
        reinterpret_cast<float2*>(p)[i] = make_float2(x, y);
    }
    __device__ __forceinline__ static void ld3(const float* p, int64_t i, float& x, float& y, float& z) {
        const float4 v = reinterpret_cast<const float4*>(p)[i];
        x = v.x;
        y = v.y;
        z = v.z;
    }
    __device__ __forceinline__ static void st3(float* p, int64_t i, float x, float y, float z) {
        reinterpret_cast<float4*>(p)[i] = make_float4(x, y, z, 0.0f);
    }
};

template <> struct Store<bf16s> {
    using C = float;
    __device__ __forceinline__ static float ld1(const bf16s* p, int64_t i) { return bf2f(p[i].b); }
    __device__ __forceinline__ static void st1(bf16s* p, int64_t i, float v) { p[i].b = f2bf(v); }
    __device__ __forceinline__ static void ld2(const bf16s* p, int64_t i, float& x, float& y) {
        const uint32_t v = reinterpret_cast<const uint32_t*>(p)[i];
        x = bf2f((uint16_t)(v & 0xFFFFu));
        y = bf2f((uint16_t)(v >> 16));
    }
    __device__ __forceinline__ static void st2(bf16s* p, int64_t i, float x, float y) {
        reinterpret_cast<uint32_t*>(p)[i] = (uint32_t)f2bf(x) | ((uint32_t)f2bf(y) << 16);
    }
    __device__ __forceinline__ static void ld3(const bf16s* p, int64_t i, float& x, float& y, float& z) {
        const uint2 v = reinterpret_cast<const uint2*>(p)[i];
        x = bf2f((uint16_t)(v.x & 0xFFFFu));
        y = bf2f((uint16_t)(v.x >> 16));
        z = bf2f((uint16_t)(v.y & 0xFFFFu));
    }
    __device__ __forceinline__ static void st3(bf16s* p, int64_t i, float x, float y, float z) {
        reinterpret_cast<uint2*>(p)[i] = make_uint2((uint32_t)f2bf(x) | ((uint32_t)f2bf(y) << 16), (uint32_t)f2bf(z));
    }
};

// Packed weights and stencil positions are streamed once per half step:
// load them non-temporally so that they do not displace the gathered field
// values in L2.
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));

// Position of value u (0..3) of lane `lane` in a packed weight chunk block of
// 64 lanes x 4 values.  FP32 is lane-major ([64][4]: one 16-byte load per
// lane, a contiguous 1 KB per wavefront); FP64 is split into two halves
// ([2][64][2]) so that each of a lane's two 16-byte loads is also part of one
// contiguous 1 KB run per wavefront (lane-major FP64 would give each load a
// 32-byte lane stride, touching every cache line of the block twice).
template <typename TW>
struct WChunk {
    static constexpr int LS = 4;  // values between consecutive lanes
    __host__ __device__ static constexpr int at(int lane, int u) { return lane * 4 + u; }
};
template <>
struct WChunk<double> {
    static constexpr int LS = 2;
    __host__ __device__ static constexpr int at(int lane, int u) { return (u >> 1) * 128 + lane * 2 + (u & 1); }
};

// the four packed weights of a chunk at p (the block base plus lane * LS)
__device__ __forceinline__ void ldw4(const float* p, float (&w)[4]) {
    const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
    w[0] = v.x;
    w[1] = v.y;
    w[2] = v.z;
    w[3] = v.w;
}
__device__ __forceinline__ void ldw4(const double* p, double (&w)[4]) {
    const nt_d2 a = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    const nt_d2 b = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p + 128));
    w[0] = a.x;
    w[1] = a.y;
    w[2] = b.x;
    w[3] = b.y;
}
// plain (cached) loads for the global-gather kernels, whose weight stream
// competes less with the L2-resident gathers than with the staged halo copies
__device__ __forceinline__ void ldw4p(const float* p, float (&w)[4]) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    w[0] = v.x;
    w[1] = v.y;
    w[2] = v.z;
    w[3] = v.w;
}
__device__ __forceinline__ void ldw4p(const double* p, double (&w)[4]) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 128);
    w[0] = a.x;
    w[1] = a.y;
    w[2] = b.x;
    w[3] = b.y;
}
__device__ __forceinline__ uint4 ldu4s(const uint4* p) {
    const nt_u4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int idx4(const int4& j, int u) {
    return u == 0 ? j.x : (u == 1 ? j.y : (u == 2 ? j.z : j.w));
}
