// Packed weight chunks: how the step kernels store and read the weights of
// 4 consecutive stencil slots of one lane.
//
// FP32: the 4 values, lane-major ([tile][chunk][64][4]), one 16-byte load
// per lane; FP64: the 4 values in two halves ([tile][chunk][2][64][2]), two
// 16-byte loads per lane, each reading a contiguous 1 KB per wavefront.
//
// W22 (compressed FP32 weights): 12 bytes per chunk -- four 22-bit signed
// integer mantissas m_u and one 8-bit exponent b shared by the chunk; the
// weight is m_u 2^(b - 127), decoded exactly in FP32.  The exponent is that
// of the chunk's largest |w| plus one, less 21, so the largest mantissa
// keeps 21 significant bits and smaller weights keep the same absolute step
// (2^(b - 127)).  Words are stored word-major within a tile's chunk
// ([tile][chunk][3][64]) so each of a wavefront's three dword loads reads one
// contiguous 256-byte run.  Bit layout of the three words:
//   w0 = m0[21:0] | m3[9:0]   << 22
//   w1 = m1[21:0] | m3[19:10] << 22
//   w2 = m2[21:0] | m3[21:20] << 22 | b << 24
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fields.h"
#include "../../include/rbffd.h"

struct w22 {
    uint32_t v;
};

template <typename TW>
struct WF {
    using V = TW;                      // value type the kernels compute with
    static constexpr int CH = 256;     // TW elements per (tile, chunk) block
    static constexpr int LS = WChunk<TW>::LS;  // TW elements between consecutive lanes
    __device__ __forceinline__ static void ld(const TW* p, V (&w)[4]) { ldw4(p, w); }
    __device__ __forceinline__ static void ldp(const TW* p, V (&w)[4]) { ldw4p(p, w); }
    __device__ __forceinline__ static void store(TW* p, const double (&w)[4]) {
        for (int u = 0; u < 4; ++u) p[WChunk<TW>::at(0, u)] = (TW)w[u];
    }
};

__device__ __forceinline__ int32_t sext22(uint32_t x) { return ((int32_t)(x << 10)) >> 10; }

__device__ __forceinline__ void w22_decode(uint32_t w0, uint32_t w1, uint32_t w2, float (&w)[4]) {
    const float sc = __uint_as_float((w2 >> 24) << 23);
    const uint32_t m3 = (w0 >> 22) | ((w1 >> 22) << 10) | (((w2 >> 22) & 3u) << 20);
    w[0] = (float)sext22(w0) * sc;
    w[1] = (float)sext22(w1) * sc;
    w[2] = (float)sext22(w2) * sc;
    w[3] = (float)sext22(m3) * sc;
}

template <>
struct WF<w22> {
    using V = float;
    static constexpr int CH = 3 * 64;
    static constexpr int LS = 1;
    __device__ __forceinline__ static void ld(const w22* p, float (&w)[4]) {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
        w22_decode(__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 64),
                   __builtin_nontemporal_load(q + 128), w);
    }
    __device__ __forceinline__ static void ldp(const w22* p, float (&w)[4]) {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
        w22_decode(q[0], q[64], q[128], w);
    }
    // encode 4 FP64 weights (rounded to nearest, ties to even)
    __device__ __forceinline__ static void store(w22* p, const double (&w)[4]) {
        double mx = 0.0;
        for (int u = 0; u < 4; ++u) mx = fmax(mx, fabs(w[u]));
        int e = 0;
        if (mx > 0.0) frexp(mx, &e);      // 2^(e-1) <= mx < 2^e
        int b = e - 21 + 127;             // |w| / 2^(b-127) < 2^21
        b = b < 1 ? 1 : (b > 254 ? 254 : b);
        uint32_t m[4];
        for (int u = 0; u < 4; ++u) {
            double q = rint(ldexp(w[u], 127 - b));
            q = fmin(fmax(q, -2097152.0), 2097151.0);
            m[u] = (uint32_t)(int32_t)q & 0x3FFFFFu;
        }
        uint32_t* o = reinterpret_cast<uint32_t*>(p);
        o[0] = m[0] | ((m[3] & 0x3FFu) << 22);
        o[64] = m[1] | (((m[3] >> 10) & 0x3FFu) << 22);
        o[128] = m[2] | (((m[3] >> 20) & 0x3u) << 22) | ((uint32_t)b << 24);
    }
};

// bytes of one lane's chunk in the arena
inline int chunk_bytes(int wdtype) { return wdtype == RBFFD_F64 ? 32 : (wdtype == RBFFD_W22 ? 12 : 16); }
