// K independent fields sharing one weight set (2D TMz, collocated, FP32).
// Fields are stored [N][F][K] (K contiguous).  Three kernel designs:
//
// * global gathers (k_hb, k_eb): a wavefront owns one node and 64
//   consecutive fields; the node's stencil indices and weights are
//   wave-uniform (scalar loads, read once for all 64 fields) and every
//   neighbour gather is one contiguous 256-byte row.  The grid is
//   persistent: a fixed number of resident workgroups strides over (node,
//   field-chunk) items.
// * LDS-staged, one (tile, field-slice) item per workgroup (k_hbl, k_ebl).
// * LDS-staged and persistent, with staging wavefronts that fill a second
//   LDS buffer while the others sum (k_bpers).
//
// The update is the eq. 19 step of the single-field kernels (Kolar-Pozun &
// Kosec, arXiv 2508.18205, Section 5) with every operator summed as eq. 16
// writes it, over the whole stencil with the centre's own weight, rather than
// in the single-field kernels' difference form: a batch is bound by its
// arithmetic, not by memory, and this form needs one FMA per weight and
// field where the difference form needs a subtraction as well.
#include <algorithm>
#include "common.h"

namespace {

struct BA {
    const float* E;
    const float* H;
    float* out;
    const int32_t* idx;   // [N][S]
    const float* wc;      // [N][2][C]
    const float* wh;      // [N][V]
    const float* w0;      // [N][4] centre weights (curl x, curl y, hyperviscosity)
    int64_t N;
    int K, KC;            // fields, 64-field chunks
    int S, C, V;          // padded slot counts (multiples of 4)
    float a;
    const float* gk;      // per-field gamma [K]
    const uint8_t* emask;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__global__ __launch_bounds__(256) void k_hb(BA a) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int w0 = uni((int)blockIdx.x * wpb + (int)(threadIdx.x >> 6));
    const int nw = (int)gridDim.x * wpb;
    const int64_t items = a.N * a.KC;
    for (int64_t it = w0; it < items; it += nw) {
        const int64_t i = it / a.KC;
        const int k = (int)(it % a.KC) * 64 + lane;
        const bool on = k < a.K;
        const int kk = on ? k : a.K - 1;
        const int K = a.K;
        const float e0 = a.E[i * K + kk];
        const float hx0 = a.H[(i * 2 + 0) * K + kk], hy0 = a.H[(i * 2 + 1) * K + kk];
        const float G = a.gk[kk];
        const float* c0 = a.w0 + i * 4;
        float dx = c0[0] * e0, dy = c0[1] * e0, vx = c0[2] * hx0, vy = c0[2] * hy0;
        const int32_t* pi = a.idx + i * a.S;
        const float* px = a.wc + (i * 2 + 0) * a.C;
        const float* py = a.wc + (i * 2 + 1) * a.C;
        const float* ph = a.wh + i * a.V;
        const int both = min(a.C, a.V);
        int s = 0;
        for (; s < both; ++s) {
            const int64_t j = pi[s];
            const float e = a.E[j * K + kk];
            dx += px[s] * e;
            dy += py[s] * e;
            vx += ph[s] * a.H[(j * 2 + 0) * K + kk];
            vy += ph[s] * a.H[(j * 2 + 1) * K + kk];
        }
        for (; s < a.C; ++s) {
            const int64_t j = pi[s];
            const float e = a.E[j * K + kk];
            dx += px[s] * e;
            dy += py[s] * e;
        }
        for (; s < a.V; ++s) {
            const int64_t j = pi[s];
            vx += ph[s] * a.H[(j * 2 + 0) * K + kk];
            vy += ph[s] * a.H[(j * 2 + 1) * K + kk];
        }
        if (on) {
            a.out[(i * 2 + 0) * K + k] = hx0 + a.a * (-dy + G * vx);
            a.out[(i * 2 + 1) * K + k] = hy0 + a.a * (dx + G * vy);
        }
    }
}

__global__ __launch_bounds__(256) void k_eb(BA a) {
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int w0 = uni((int)blockIdx.x * wpb + (int)(threadIdx.x >> 6));
    const int nw = (int)gridDim.x * wpb;
    const int64_t items = a.N * a.KC;
    for (int64_t it = w0; it < items; it += nw) {
        const int64_t i = it / a.KC;
        const int k = (int)(it % a.KC) * 64 + lane;
        const bool on = k < a.K;
        const int kk = on ? k : a.K - 1;
        const int K = a.K;
        const float e0 = a.E[i * K + kk];
        const float hx0 = a.H[(i * 2 + 0) * K + kk], hy0 = a.H[(i * 2 + 1) * K + kk];
        const float G = a.gk[kk];
        const float* c0 = a.w0 + i * 4;
        // curl H = D^dx Hy - D^dy Hx
        float cu = c0[0] * hy0, ve = c0[2] * e0;
        cu -= c0[1] * hx0;
        const int32_t* pi = a.idx + i * a.S;
        const float* px = a.wc + (i * 2 + 0) * a.C;
        const float* py = a.wc + (i * 2 + 1) * a.C;
        const float* ph = a.wh + i * a.V;
        const int both = min(a.C, a.V);
        int s = 0;
        for (; s < both; ++s) {
            const int64_t j = pi[s];
            cu += px[s] * a.H[(j * 2 + 1) * K + kk];
            cu -= py[s] * a.H[(j * 2 + 0) * K + kk];
            ve += ph[s] * a.E[j * K + kk];
        }
        for (; s < a.C; ++s) {
            const int64_t j = pi[s];
            cu += px[s] * a.H[(j * 2 + 1) * K + kk];
            cu -= py[s] * a.H[(j * 2 + 0) * K + kk];
        }
        for (; s < a.V; ++s) {
            const int64_t j = pi[s];
            ve += ph[s] * a.E[j * K + kk];
        }
        if (on) a.out[i * K + k] = (a.emask[i] & 1) ? e0 + a.a * (cu + G * ve) : 0.f;
    }
}

// ---- LDS-staged batch -----------------------------------------------------
// Workgroup = one 128-node tile x one 16-field slice (512 threads; the halo
// slice takes ~60 KB of LDS, so two workgroups share a CU and one stages
// while the other sums).  It copies the slice of every halo node's rows (E,
// Hx, Hy) into LDS, then 4 threads per node each update 4 fields; stencil
// positions (16-bit) and weights come from tile-sliced packed arrays laid out
// as the single-field kernels' (halo lists built for 128-node tiles), one
// 16-byte load per 4 slots shared by the node's 4 threads, and the centre
// weights of eq. 16 from one 16-byte load per node; the node's own values
// come from its row of the staged slice.  The slices of one tile are
// consecutive workgroups, so they meet the tile's weights in L2.
struct BLA {
    const float* E;
    const float* H;
    float* out;
    const uint4* lidx;    // [tiles][Q8][64] x 8 u16 halo positions
    const uint16_t* lself;// [tiles * 64] each node's own halo position
    const int32_t* hpool;
    const int32_t* hoff;  // [128-node workgroup tiles + 1]
    const float* wc;      // [tiles][C4][2][64][4]
    const float* wh;      // [tiles][V4][64][4]
    const float* w0;      // [N][4] centre weights (curl x, curl y, hyperviscosity)
    int64_t N, tiles;
    int K, KS, C4, V4, Q8, xcd;
    int64_t items;        // (tile, slice) items
    int64_t slice;        // floats per LDS halo-slice buffer (persistent kernels)
    float a;
    const float* gk;      // per-field gamma [K]
    const uint8_t* emask;
};

struct f4 {
    float x, y, z, w;
};
__device__ __forceinline__ f4 ldf4(const float* p) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    return {v.x, v.y, v.z, v.w};
}
// the halo rows are streamed once per item: non-temporal loads keep them from
// displacing the tile's weights, which the tile's other slices read from L2
typedef float ntf4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4 ldf4nt(const float* p) {
    const ntf4_t v = __builtin_nontemporal_load(reinterpret_cast<const ntf4_t*>(p));
    return {v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ void stf4(float* p, const f4& v) {
    *reinterpret_cast<float4*>(p) = make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void fma4(f4& acc, float w, const f4& a) {
    acc.x += w * a.x;
    acc.y += w * a.y;
    acc.z += w * a.z;
    acc.w += w * a.w;
}
__device__ __forceinline__ void fms4(f4& acc, float w, const f4& a) {
    acc.x -= w * a.x;
    acc.y -= w * a.y;
    acc.z -= w * a.z;
    acc.w -= w * a.w;
}
__device__ __forceinline__ f4 mul4(float w, const f4& a) { return {w * a.x, w * a.y, w * a.z, w * a.w}; }
__device__ __forceinline__ int posq(const uint4& v, int half, int u) {
    const uint32_t w = half ? (u < 2 ? v.z : v.w) : (u < 2 ? v.x : v.y);
    return (int)((u & 1) ? (w >> 16) : (w & 0xFFFFu));
}

// The slice of every halo node's rows (E, Hx, Hy) into LDS, laid out
// [k][c][KSL].  Thread t of nt (the whole workgroup, or its staging
// wavefronts; nt a multiple of the Q 16-byte pieces per row) copies piece
// q = t % Q of the three rows of halo nodes t / Q, t / Q + nt / Q, ...; each
// round it loads the list values of NB nodes, then their 3 NB pieces, then
// stores them, so that the loads are in flight together.
template <int KSL>
__device__ __forceinline__ void stage_slice(const BLA& a, float* sm, int64_t tile, int ks, int t, int nt) {
    constexpr int Q = KSL / 4;
    constexpr int NB = 3;
    const int h0 = a.hoff[tile], hc = a.hoff[tile + 1] - h0;
    const uint64_t K = (uint32_t)a.K;
    const int q = t & (Q - 1), step = nt / Q;
    const float* E = a.E + ks * KSL + q * 4;
    const float* H = a.H + ks * KSL + q * 4;
    float* dst = sm + q * 4;
    for (int base = t / Q; base < hc; base += NB * step) {
        int j[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int k = base + b * step;
            j[b] = k < hc ? a.hpool[h0 + k] : -1;
        }
        f4 v[NB][3];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (j[b] < 0) continue;
            const uint64_t r = (uint32_t)j[b];
            if constexpr (KSL == 16) {
                v[b][0] = ldf4nt(E + r * K);
                v[b][1] = ldf4nt(H + 2 * r * K);
                v[b][2] = ldf4nt(H + (2 * r + 1) * K);
            } else {
                // narrower slices share 64-byte segments with the next
                // slice's pieces, which find them in L2
                v[b][0] = ldf4(E + r * K);
                v[b][1] = ldf4(H + 2 * r * K);
                v[b][2] = ldf4(H + (2 * r + 1) * K);
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (j[b] < 0) continue;
            float* d = dst + (base + b * step) * 3 * KSL;
            stf4(d, v[b][0]);
            stf4(d + KSL, v[b][1]);
            stf4(d + 2 * KSL, v[b][2]);
        }
    }
}

// One 4-slot chunk of a node's stencil: the halo values it reads from LDS
// and its weights, all read before the chunk is summed so that the LDS reads
// of a chunk are in flight together.
struct HChunk {
    f4 e[4], x[4], y[4];
    f4 wx, wy, wh;
};
struct EChunk {
    f4 hx[4], hy[4], e[4];
    f4 wx, wy, wh;
};

template <int KSL>
__device__ __forceinline__ const float* row(const float* sm, int k, int c, int fq) {
    return sm + (k * 3 + c) * KSL + fq * 4;
}

// the weights of chunk q (left as they are past the chunk counts)
__device__ __forceinline__ void w_read(const BLA& a, int q, const float* pc, const float* ph, f4& wx, f4& wy, f4& wh) {
    if (q < a.C4) {
        wx = ldf4(pc + (q * 2 + 0) * RBFFD_TILE * 4);
        wy = ldf4(pc + (q * 2 + 1) * RBFFD_TILE * 4);
    }
    if (q < a.V4) wh = ldf4(ph + q * RBFFD_TILE * 4);
}

template <int KSL>
__device__ __forceinline__ void h_read(const BLA& a, const float* sm, uint4 lp, int q, int fq, HChunk& c) {
    const int hf = q & 1;
    if (q < a.C4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) c.e[u] = ldf4(row<KSL>(sm, posq(lp, hf, u), 0, fq));
    }
    if (q < a.V4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = posq(lp, hf, u);
            c.x[u] = ldf4(row<KSL>(sm, k, 1, fq));
            c.y[u] = ldf4(row<KSL>(sm, k, 2, fq));
        }
    }
}

__device__ __forceinline__ void h_sum(const BLA& a, int q, const HChunk& c, f4& dx, f4& dy, f4& vx, f4& vy) {
    if (q < a.C4) {
        const float wxs[4] = {c.wx.x, c.wx.y, c.wx.z, c.wx.w}, wys[4] = {c.wy.x, c.wy.y, c.wy.z, c.wy.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            fma4(dx, wxs[u], c.e[u]);
            fma4(dy, wys[u], c.e[u]);
        }
    }
    if (q < a.V4) {
        const float whs[4] = {c.wh.x, c.wh.y, c.wh.z, c.wh.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            fma4(vx, whs[u], c.x[u]);
            fma4(vy, whs[u], c.y[u]);
        }
    }
}

template <int KSL>
__device__ __forceinline__ void e_read(const BLA& a, const float* sm, uint4 lp, int q, int fq, EChunk& c) {
    const int hf = q & 1;
    if (q < a.C4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = posq(lp, hf, u);
            c.hx[u] = ldf4(row<KSL>(sm, k, 1, fq));
            c.hy[u] = ldf4(row<KSL>(sm, k, 2, fq));
        }
    }
    if (q < a.V4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) c.e[u] = ldf4(row<KSL>(sm, posq(lp, hf, u), 0, fq));
    }
}

__device__ __forceinline__ void e_sum(const BLA& a, int q, const EChunk& c, f4& cu, f4& ve) {
    if (q < a.C4) {
        const float wxs[4] = {c.wx.x, c.wx.y, c.wx.z, c.wx.w}, wys[4] = {c.wy.x, c.wy.y, c.wy.z, c.wy.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            // curl H = D^dx Hy - D^dy Hx
            fma4(cu, wxs[u], c.hy[u]);
            fms4(cu, wys[u], c.hx[u]);
        }
    }
    if (q < a.V4) {
        const float whs[4] = {c.wh.x, c.wh.y, c.wh.z, c.wh.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) fma4(ve, whs[u], c.e[u]);
    }
}

// A chunk with both curl and hyperviscosity slots: its twelve LDS reads are
// issued together, then summed (no per-part branches, so that the reads of
// one chunk are all in flight before the first sum waits).
template <int KSL, int HF>
__device__ __forceinline__ void h_read_full(const float* sm, uint4 lp, int fq, HChunk& c) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = posq(lp, HF, u);
        c.e[u] = ldf4(row<KSL>(sm, k, 0, fq));
        c.x[u] = ldf4(row<KSL>(sm, k, 1, fq));
        c.y[u] = ldf4(row<KSL>(sm, k, 2, fq));
    }
}

__device__ __forceinline__ void h_sum_full(const HChunk& c, const f4& wx, const f4& wy, const f4& wh, f4& dx, f4& dy,
                                           f4& vx, f4& vy) {
    const float wxs[4] = {wx.x, wx.y, wx.z, wx.w}, wys[4] = {wy.x, wy.y, wy.z, wy.w};
    const float whs[4] = {wh.x, wh.y, wh.z, wh.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        fma4(dx, wxs[u], c.e[u]);
        fma4(dy, wys[u], c.e[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        fma4(vx, whs[u], c.x[u]);
        fma4(vy, whs[u], c.y[u]);
    }
}

template <int KSL, int HF>
__device__ __forceinline__ void e_read_full(const float* sm, uint4 lp, int fq, EChunk& c) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = posq(lp, HF, u);
        c.hx[u] = ldf4(row<KSL>(sm, k, 1, fq));
        c.hy[u] = ldf4(row<KSL>(sm, k, 2, fq));
        c.e[u] = ldf4(row<KSL>(sm, k, 0, fq));
    }
}

__device__ __forceinline__ void e_sum_full(const EChunk& c, const f4& wx, const f4& wy, const f4& wh, f4& cu, f4& ve) {
    const float wxs[4] = {wx.x, wx.y, wx.z, wx.w}, wys[4] = {wy.x, wy.y, wy.z, wy.w};
    const float whs[4] = {wh.x, wh.y, wh.z, wh.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        fma4(cu, wxs[u], c.hy[u]);
        fms4(cu, wys[u], c.hx[u]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) fma4(ve, whs[u], c.e[u]);
}

// Chunks with hyperviscosity slots only (past the curl stencil): their LDS
// reads and sums, and a branch-free loop over their pairs from an even chunk.
template <int KSL, int HF>
__device__ __forceinline__ void hv_h(const float* sm, uint4 lp, int fq, const f4& wh, f4& vx, f4& vy) {
    f4 x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = posq(lp, HF, u);
        x[u] = ldf4(row<KSL>(sm, k, 1, fq));
        y[u] = ldf4(row<KSL>(sm, k, 2, fq));
    }
    const float whs[4] = {wh.x, wh.y, wh.z, wh.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        fma4(vx, whs[u], x[u]);
        fma4(vy, whs[u], y[u]);
    }
}
template <int KSL, int HF>
__device__ __forceinline__ void hv_e(const float* sm, uint4 lp, int fq, const f4& wh, f4& ve) {
    f4 e[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) e[u] = ldf4(row<KSL>(sm, posq(lp, HF, u), 0, fq));
    const float whs[4] = {wh.x, wh.y, wh.z, wh.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) fma4(ve, whs[u], e[u]);
}

// H update of one (tile, slice) item from its staged halo slice sm, by
// thread tid of the tile's RBFFD_WGT_BATCH * TPN
template <int TPN>
__device__ __forceinline__ void h_item(const BLA& a, const float* sm, int64_t tile, int ks, int tid) {
    constexpr int KSL = 4 * TPN;          // fields per slice, 4 per thread
    const int nl = tid / TPN, fq = tid % TPN;
    const int64_t i = tile * RBFFD_WGT_BATCH + nl;
    if (i >= a.N) return;
    const int64_t t64 = i / RBFFD_TILE;
    const int ln = (int)(i % RBFFD_TILE);
    const int64_t K = a.K;
    const int k0 = ks * KSL + fq * 4;
    // the node's own values, from its row of the staged slice
    const int sp = a.lself[i];
    const f4 e0 = ldf4(row<KSL>(sm, sp, 0, fq)), hx0 = ldf4(row<KSL>(sm, sp, 1, fq)), hy0 = ldf4(row<KSL>(sm, sp, 2, fq));
    // the centre's own terms of eq. 16 first
    const f4 c0 = ldf4(a.w0 + i * 4);
    f4 dx = mul4(c0.x, e0), dy = mul4(c0.y, e0), vx = mul4(c0.z, hx0), vy = mul4(c0.z, hy0);
    const uint4* pl = a.lidx + t64 * a.Q8 * RBFFD_TILE + ln;
    const float* pc = a.wc + (t64 * a.C4 * 2 * RBFFD_TILE + ln) * 4;
    const float* ph = a.wh + (t64 * a.V4 * RBFFD_TILE + ln) * 4;
    const int qm = max(a.C4, a.V4), qb = min(a.C4, a.V4);
    const int np = (qm + 1) >> 1;
    HChunk A;
    // chunk pairs in which every chunk has both parts: the weights of the
    // next chunk and the positions of the next pair are loaded while the
    // current chunk is read from LDS and summed (indices clamped to the last
    // chunk and pair, so the loads need no branch)
    int q = 0;
    {
        f4 wx0 = ldf4(pc), wy0 = ldf4(pc + RBFFD_TILE * 4), wh0 = ldf4(ph);
        uint4 lp = pl[0];
        for (; q + 2 <= qb; q += 2) {
            const uint4 lpn = pl[min((q >> 1) + 1, np - 1) * RBFFD_TILE];
            const f4 wx1 = ldf4(pc + ((q + 1) * 2 + 0) * RBFFD_TILE * 4);
            const f4 wy1 = ldf4(pc + ((q + 1) * 2 + 1) * RBFFD_TILE * 4);
            const f4 wh1 = ldf4(ph + (q + 1) * RBFFD_TILE * 4);
            h_read_full<KSL, 0>(sm, lp, fq, A);
            h_sum_full(A, wx0, wy0, wh0, dx, dy, vx, vy);
            const int qc = min(q + 2, a.C4 - 1), qv = min(q + 2, a.V4 - 1);
            wx0 = ldf4(pc + (qc * 2 + 0) * RBFFD_TILE * 4);
            wy0 = ldf4(pc + (qc * 2 + 1) * RBFFD_TILE * 4);
            wh0 = ldf4(ph + qv * RBFFD_TILE * 4);
            h_read_full<KSL, 1>(sm, lp, fq, A);
            h_sum_full(A, wx1, wy1, wh1, dx, dy, vx, vy);
            lp = lpn;
        }
    }
    // pairs of hyperviscosity-only chunks, then the rest: an odd chunk with
    // both parts, or the chunks past the shorter part
    if (q == qb && !(q & 1) && a.V4 > a.C4) {
        for (; q + 2 <= a.V4; q += 2) {
            const uint4 lp = pl[(q >> 1) * RBFFD_TILE];
            const f4 w0 = ldf4(ph + q * RBFFD_TILE * 4), w1 = ldf4(ph + (q + 1) * RBFFD_TILE * 4);
            hv_h<KSL, 0>(sm, lp, fq, w0, vx, vy);
            hv_h<KSL, 1>(sm, lp, fq, w1, vx, vy);
        }
    }
    for (; q < qm; ++q) {
        f4 zx{0, 0, 0, 0}, zy{0, 0, 0, 0}, zh{0, 0, 0, 0};
        w_read(a, q, pc, ph, zx, zy, zh);
        A.wx = zx;
        A.wy = zy;
        A.wh = zh;
        const uint4 lp = pl[(q >> 1) * RBFFD_TILE];
        h_read<KSL>(a, sm, lp, q, fq, A);
        h_sum(a, q, A, dx, dy, vx, vy);
    }
    const float Af = a.a;
    const f4 G = ldf4(a.gk + k0);
    stf4(a.out + (i * 2) * K + k0, {hx0.x + Af * (-dy.x + G.x * vx.x), hx0.y + Af * (-dy.y + G.y * vx.y),
                                    hx0.z + Af * (-dy.z + G.z * vx.z), hx0.w + Af * (-dy.w + G.w * vx.w)});
    stf4(a.out + (i * 2 + 1) * K + k0, {hy0.x + Af * (dx.x + G.x * vy.x), hy0.y + Af * (dx.y + G.y * vy.y),
                                        hy0.z + Af * (dx.z + G.z * vy.z), hy0.w + Af * (dx.w + G.w * vy.w)});
}

// E update of one (tile, slice) item (as h_item)
template <int TPN>
__device__ __forceinline__ void e_item(const BLA& a, const float* sm, int64_t tile, int ks, int tid) {
    constexpr int KSL = 4 * TPN;
    const int nl = tid / TPN, fq = tid % TPN;
    const int64_t i = tile * RBFFD_WGT_BATCH + nl;
    if (i >= a.N) return;
    const int64_t t64 = i / RBFFD_TILE;
    const int ln = (int)(i % RBFFD_TILE);
    const int64_t K = a.K;
    const int k0 = ks * KSL + fq * 4;
    // the node's own values, from its row of the staged slice
    const int sp = a.lself[i];
    const f4 e0 = ldf4(row<KSL>(sm, sp, 0, fq)), hx0 = ldf4(row<KSL>(sm, sp, 1, fq)), hy0 = ldf4(row<KSL>(sm, sp, 2, fq));
    const f4 c0 = ldf4(a.w0 + i * 4);
    f4 cu = mul4(c0.x, hy0), ve = mul4(c0.z, e0);
    fms4(cu, c0.y, hx0);
    const uint4* pl = a.lidx + t64 * a.Q8 * RBFFD_TILE + ln;
    const float* pc = a.wc + (t64 * a.C4 * 2 * RBFFD_TILE + ln) * 4;
    const float* ph = a.wh + (t64 * a.V4 * RBFFD_TILE + ln) * 4;
    const int qm = max(a.C4, a.V4), qb = min(a.C4, a.V4);
    const int np = (qm + 1) >> 1;
    EChunk A;
    int q = 0;
    {
        f4 wx0 = ldf4(pc), wy0 = ldf4(pc + RBFFD_TILE * 4), wh0 = ldf4(ph);
        uint4 lp = pl[0];
        for (; q + 2 <= qb; q += 2) {
            const uint4 lpn = pl[min((q >> 1) + 1, np - 1) * RBFFD_TILE];
            const f4 wx1 = ldf4(pc + ((q + 1) * 2 + 0) * RBFFD_TILE * 4);
            const f4 wy1 = ldf4(pc + ((q + 1) * 2 + 1) * RBFFD_TILE * 4);
            const f4 wh1 = ldf4(ph + (q + 1) * RBFFD_TILE * 4);
            e_read_full<KSL, 0>(sm, lp, fq, A);
            e_sum_full(A, wx0, wy0, wh0, cu, ve);
            const int qc = min(q + 2, a.C4 - 1), qv = min(q + 2, a.V4 - 1);
            wx0 = ldf4(pc + (qc * 2 + 0) * RBFFD_TILE * 4);
            wy0 = ldf4(pc + (qc * 2 + 1) * RBFFD_TILE * 4);
            wh0 = ldf4(ph + qv * RBFFD_TILE * 4);
            e_read_full<KSL, 1>(sm, lp, fq, A);
            e_sum_full(A, wx1, wy1, wh1, cu, ve);
            lp = lpn;
        }
    }
    if (q == qb && !(q & 1) && a.V4 > a.C4) {
        for (; q + 2 <= a.V4; q += 2) {
            const uint4 lp = pl[(q >> 1) * RBFFD_TILE];
            const f4 w0 = ldf4(ph + q * RBFFD_TILE * 4), w1 = ldf4(ph + (q + 1) * RBFFD_TILE * 4);
            hv_e<KSL, 0>(sm, lp, fq, w0, ve);
            hv_e<KSL, 1>(sm, lp, fq, w1, ve);
        }
    }
    for (; q < qm; ++q) {
        f4 zx{0, 0, 0, 0}, zy{0, 0, 0, 0}, zh{0, 0, 0, 0};
        w_read(a, q, pc, ph, zx, zy, zh);
        A.wx = zx;
        A.wy = zy;
        A.wh = zh;
        const uint4 lp = pl[(q >> 1) * RBFFD_TILE];
        e_read<KSL>(a, sm, lp, q, fq, A);
        e_sum(a, q, A, cu, ve);
    }
    const float Af = a.a;
    const f4 G = ldf4(a.gk + k0);
    const bool keep = a.emask[i] & 1;
    stf4(a.out + i * K + k0, keep ? f4{e0.x + Af * (cu.x + G.x * ve.x), e0.y + Af * (cu.y + G.y * ve.y),
                                       e0.z + Af * (cu.z + G.z * ve.z), e0.w + Af * (cu.w + G.w * ve.w)}
                                  : f4{0, 0, 0, 0});
}

// one item per workgroup: the whole workgroup stages the halo slice, then sums
template <int TPN>
__global__ __launch_bounds__(RBFFD_WGT_BATCH * TPN) void k_hbl(BLA a) {
    extern __shared__ __align__(16) float sm[];
    const int wg = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int64_t tile = wg / a.KS;
    const int ks = wg % a.KS;
    stage_slice<4 * TPN>(a, sm, tile, ks, (int)threadIdx.x, (int)blockDim.x);
    __syncthreads();
    h_item<TPN>(a, sm, tile, ks, (int)threadIdx.x);
}

template <int TPN>
__global__ __launch_bounds__(RBFFD_WGT_BATCH * TPN) void k_ebl(BLA a) {
    extern __shared__ __align__(16) float sm[];
    const int wg = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int64_t tile = wg / a.KS;
    const int ks = wg % a.KS;
    stage_slice<4 * TPN>(a, sm, tile, ks, (int)threadIdx.x, (int)blockDim.x);
    __syncthreads();
    e_item<TPN>(a, sm, tile, ks, (int)threadIdx.x);
}

// ---- persistent batch with staging wavefronts ------------------------------
// A resident workgroup walks the items v, v + G, v + 2G, ... (v its
// XCD-ordered index, G the grid).  Its first RBFFD_WGT_BATCH * TPN threads
// sum item n from one LDS buffer while the last 64 * TPN threads (the
// staging wavefronts) copy the halo slice of item n + 1 into the other, so
// that the halo loads are in flight while the sums run; one barrier per item
// hands the buffers over.  Every thread makes the same number of trips
// through the loop, so every barrier is reached by the whole workgroup.
template <int TPN, bool HUPD>
__global__ __launch_bounds__(RBFFD_WGT_BATCH * TPN + 64 * TPN) void k_bpers(BLA a) {
    constexpr int NC = RBFFD_WGT_BATCH * TPN, NP = 64 * TPN;
    extern __shared__ __align__(16) float sm[];
    const int64_t n = a.items, G = gridDim.x;
    const int64_t v = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int t = (int)threadIdx.x;
    const bool prod = t >= NC;
    int b = 0;
    if (prod && v < n) stage_slice<4 * TPN>(a, sm, v / a.KS, (int)(v % a.KS), t - NC, NP);
    __syncthreads();
    for (int64_t it = v; it < n; it += G) {
        float* cur = sm + (int64_t)b * a.slice;
        if (prod) {
            const int64_t nx = it + G;
            if (nx < n) stage_slice<4 * TPN>(a, sm + (int64_t)(b ^ 1) * a.slice, nx / a.KS, (int)(nx % a.KS), t - NC, NP);
        } else if (HUPD) {
            h_item<TPN>(a, cur, it / a.KS, (int)(it % a.KS), t);
        } else {
            e_item<TPN>(a, cur, it / a.KS, (int)(it % a.KS), t);
        }
        __syncthreads();
        b ^= 1;
    }
}

BA make_args(const rbffd_plan* p) {
    const OpBlock& o = p->opH;
    BA a{};
    a.idx = o.bidx;
    a.wc = o.bwc;
    a.wh = o.bwh;
    a.w0 = o.bw0;
    a.N = o.Nt;
    a.K = p->K;
    a.KC = (int)cdiv(p->K, 64);
    a.S = o.S4 * 4;
    a.C = o.C4 * 4;
    a.V = o.V4 * 4;
    a.gk = p->gk;
    a.emask = p->E.emask;
    return a;
}

// slice width: 16 fields (4 threads per node) when the variant asks for it
// (persist >= 16) and two workgroups' halo slices fit one CU's LDS (with one
// workgroup per CU the 8-field slices are faster), 4 fields (one thread per
// node, the smallest LDS footprint: more resident workgroups) for persist < 8,
// else 8 (2 threads per node).  The persistent kernels (lds = 2) hold two
// slices per workgroup.
int slice_tpn(const rbffd_plan* p) {
    if (!p->var.lds || p->opH.hmax <= 0) return 0;
    const bool pers = p->var.lds == 2;
    const int64_t row = (int64_t)p->opH.hmax * 3 * 4;   // LDS bytes per field of a halo slice
    auto fits = [&](int ksl) {
        if (pers || ksl == 16) return 2 * row * ksl <= RBFFD_LDS_CU;
        return row * ksl <= RBFFD_LDS_BUDGET_BATCH;
    };
    if (p->var.persist >= 16 && p->K % 16 == 0 && fits(16)) return 4;
    if (p->var.persist < 8 && p->K % 4 == 0 && fits(4)) return 1;
    if (p->K % 8 == 0 && fits(8)) return 2;
    if (p->K % 4 == 0 && fits(4)) return 1;
    return 0;
}

bool staged(const rbffd_plan* p) { return slice_tpn(p) > 0; }

// one half step (hupd: H update from E[c], H[c] into H[o]; else E update
// from E[c], H[o] into E[o])
void launch_half_staged(const rbffd_plan* p, const rbffd_fields* f, int c, bool hupd, hipStream_t st) {
    const int o = 1 - c;
    const OpBlock& ob = p->opH;
    const int tpn = slice_tpn(p);
    const int ksl = 4 * tpn;
    BLA a{};
    a.lidx = (const uint4*)ob.lidx;
    a.lself = ob.lself;
    a.hpool = ob.hpool;
    a.hoff = ob.hoff;
    a.wc = (const float*)ob.pwc;
    a.wh = (const float*)ob.pwh;
    a.w0 = ob.bw0;
    a.N = ob.Nt;
    a.tiles = ob.tiles;
    a.K = p->K;
    a.KS = p->K / ksl;
    a.C4 = ob.C4;
    a.V4 = ob.V4;
    a.Q8 = ob.Q8;
    a.xcd = p->var.xcd;
    a.gk = p->gk;
    a.emask = p->E.emask;
    a.items = ob.nwg * a.KS;
    a.slice = (int64_t)ob.hmax * 3 * ksl;
    a.E = (const float*)f->E[c];
    if (hupd) {
        a.H = (const float*)f->H[c];
        a.out = (float*)f->H[o];
        a.a = (float)(p->dt / p->p.mu0);
    } else {
        a.H = (const float*)f->H[o];
        a.out = (float*)f->E[o];
        a.a = (float)(p->dt / p->p.eps0);
    }
    if (p->var.lds == 2) {
        // persistent: as many resident workgroups as the CUs' LDS and
        // thread slots hold, never more than there are items
        const size_t lds = 2 * (size_t)a.slice * sizeof(float);
        const int threads = (RBFFD_WGT_BATCH + 64) * tpn;
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(RBFFD_LDS_CU / (int64_t)lds, 2048 / threads));
        const dim3 grid((unsigned)std::min<int64_t>(a.items, cus * per_cu)), block(threads);
        if (tpn == 4) {
            if (hupd) hipLaunchKernelGGL((k_bpers<4, true>), grid, block, lds, st, a);
            else hipLaunchKernelGGL((k_bpers<4, false>), grid, block, lds, st, a);
        } else if (tpn == 2) {
            if (hupd) hipLaunchKernelGGL((k_bpers<2, true>), grid, block, lds, st, a);
            else hipLaunchKernelGGL((k_bpers<2, false>), grid, block, lds, st, a);
        } else {
            if (hupd) hipLaunchKernelGGL((k_bpers<1, true>), grid, block, lds, st, a);
            else hipLaunchKernelGGL((k_bpers<1, false>), grid, block, lds, st, a);
        }
        return;
    }
    const dim3 grid((unsigned)a.items), block(RBFFD_WGT_BATCH * tpn);
    const size_t lds = (size_t)a.slice * sizeof(float);
    if (hupd) {
        if (tpn == 4) hipLaunchKernelGGL(k_hbl<4>, grid, block, lds, st, a);
        else if (tpn == 2) hipLaunchKernelGGL(k_hbl<2>, grid, block, lds, st, a);
        else hipLaunchKernelGGL(k_hbl<1>, grid, block, lds, st, a);
    } else {
        if (tpn == 4) hipLaunchKernelGGL(k_ebl<4>, grid, block, lds, st, a);
        else if (tpn == 2) hipLaunchKernelGGL(k_ebl<2>, grid, block, lds, st, a);
        else hipLaunchKernelGGL(k_ebl<1>, grid, block, lds, st, a);
    }
}

void launch_half(const rbffd_plan* p, const rbffd_fields* f, int c, bool hupd, hipStream_t st) {
    if (staged(p)) return launch_half_staged(p, f, c, hupd, st);
    const int o = 1 - c;
    BA a = make_args(p);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int wpb = p->var.block / 64;
    const int64_t need = cdiv(a.N * a.KC, wpb);
    const int grid = (int)std::min<int64_t>(need, (int64_t)cus * p->var.persist);
    a.E = (const float*)f->E[c];
    if (hupd) {
        a.H = (const float*)f->H[c];
        a.out = (float*)f->H[o];
        a.a = (float)(p->dt / p->p.mu0);
        hipLaunchKernelGGL(k_hb, dim3(grid), dim3(p->var.block), 0, st, a);
    } else {
        a.H = (const float*)f->H[o];
        a.out = (float*)f->E[o];
        a.a = (float)(p->dt / p->p.eps0);
        hipLaunchKernelGGL(k_eb, dim3(grid), dim3(p->var.block), 0, st, a);
    }
}

// ---- per-field energy (eq. 20) ---------------------------------------------
// U_k = h^2 sum_i (E_ik^2 + eta0^2 |(H^n_ik + H^{n+1}_ik) / 2|^2) for every
// field k, in FP64.  Pass 1: a wavefront reads one node's 64-field rows
// (lane = field) and strides over nodes; a workgroup's four wavefronts are
// summed in LDS into partial [block][K].  Pass 2 sums the partials of each
// field in block order.  Both passes return at once unless the step counter
// is a multiple of ``every``; the sample index is counter / every.
__global__ __launch_bounds__(256) void k_benergy1(const float* E, const float* Ha, const float* Hb, int64_t N,
                                                  int K, double wE, double wH, double* part, const int32_t* ctr,
                                                  int every) {
    if (*ctr % every) return;
    __shared__ double sh[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int k = blockIdx.y * 64 + lane;
    const int kk = k < K ? k : K - 1;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 4 + wv; i < N; i += (int64_t)gridDim.x * 4) {
        const double e = (double)E[i * K + kk];
        const double hx = 0.5 * ((double)Ha[(i * 2) * K + kk] + (double)Hb[(i * 2) * K + kk]);
        const double hy = 0.5 * ((double)Ha[(i * 2 + 1) * K + kk] + (double)Hb[(i * 2 + 1) * K + kk]);
        acc += wE * e * e + wH * (hx * hx + hy * hy);
    }
    sh[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && k < K) part[(int64_t)blockIdx.x * K + k] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

__global__ void k_benergy2(const double* part, int nb, int K, double* out, const int32_t* ctr, int every) {
    const int n = *ctr;
    if (n % every) return;
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k >= K) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)b * K + k];
    out[(int64_t)(n / every) * K + k] = s;
}

__global__ void k_bctr_set(int32_t* ctr, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = v;
}
__global__ void k_bctr_inc(int32_t* ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr += 1;
}

int energy_blocks(const rbffd_plan* p) {
    const int64_t cap = (int64_t)RED_BLOCKS * 12 / p->K;
    return (int)std::max<int64_t>(1, std::min<int64_t>(cap, std::min<int64_t>(1024, cdiv(p->E.N, 64))));
}

void launch_benergy(const rbffd_plan* p, const rbffd_fields* f, int c, double* out, RunWS& w, int every,
                    hipStream_t st) {
    const int o = 1 - c;
    const double wE = p->E.h * p->E.h;
    const double wH = p->eta0 * p->eta0 * wE;
    const int nb = energy_blocks(p);
    const int kc = (int)cdiv(p->K, 64);
    hipLaunchKernelGGL(k_benergy1, dim3(nb, kc), dim3(256), 0, st, (const float*)f->E[c], (const float*)f->H[c],
                       (const float*)f->H[o], p->E.N, p->K, wE, wH, w.part, (const int32_t*)w.ctr, every);
    hipLaunchKernelGGL(k_benergy2, dim3(kc), dim3(64), 0, st, (const double*)w.part, nb, p->K, out,
                       (const int32_t*)w.ctr, every);
}

// one full step c -> o; with an energy request the sample of step n is taken
// between the halves (E^n and both H levels are then available)
void full_step_b(const rbffd_plan* p, const rbffd_fields* f, int c, double* energy_out, int every, RunWS* w,
                 hipStream_t st) {
    launch_half(p, f, c, true, st);
    if (energy_out) launch_benergy(p, f, c, energy_out, *w, every, st);
    launch_half(p, f, c, false, st);
    if (energy_out) hipLaunchKernelGGL(k_bctr_inc, dim3(1), dim3(64), 0, st, w->ctr);
}

__global__ void k_field_gamma(float* gk, const double* c, int K, double fac, double gamma) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K) gk[k] = (float)(c ? c[k] * fac : gamma);
}

// every field from one single-field state: dst[i][comp][k] = src[i][comp]
__global__ void k_broadcast(const float* src, float* dst, int64_t rows, int K) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= rows * K) return;
    dst[g] = src[g / K];
}

}  // namespace

int fill_field_gamma(const rbffd_plan* p, const double* c_dev, hipStream_t st) {
    if (!p->gk) return RBFFD_OK;
    hipLaunchKernelGGL(k_field_gamma, dim3((unsigned)cdiv(p->K, 256)), dim3(256), 0, st, p->gk, c_dev, p->K,
                       p->hv_fac, p->gamma);
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

int batched_step(const rbffd_plan* p, rbffd_fields* f, int32_t nsteps, hipStream_t st) {
    if (f->eps_r) return set_err(p, RBFFD_ENOTSUP, "per-node eps_r is not supported for K-field batches");
    if (p->var.block > 256) return set_err(p, RBFFD_EINVAL, "K-field batches use at most 256 threads per workgroup");
    for (int s = 0; s < nsteps; ++s) {
        full_step_b(p, f, f->cur, nullptr, 1, nullptr, st);
        f->cur = 1 - f->cur;
    }
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

int batched_run(const rbffd_plan* p, rbffd_fields* f, const rbffd_run_args* a, void* ws, hipStream_t st) {
    if (a->n_src || a->n_rcv || a->ckpt)
        return set_err(p, RBFFD_ENOTSUP, "K-field batches run without sources, receivers or checkpoints");
    if (f->eps_r) return set_err(p, RBFFD_ENOTSUP, "per-node eps_r is not supported for K-field batches");
    if (p->var.block > 256) return set_err(p, RBFFD_EINVAL, "K-field batches use at most 256 threads per workgroup");
    if (a->energy_out && a->energy_every < 0) return set_err(p, RBFFD_EINVAL, "energy_every < 0");
    double* eo = (a->energy_out && a->energy_every > 0) ? a->energy_out : nullptr;
    const int every = eo ? a->energy_every : 1;
    RunWS w = run_ws(ws);
    if (eo) hipLaunchKernelGGL(k_bctr_set, dim3(1), dim3(64), 0, st, w.ctr, 0);
    int s = 0;
    if (a->use_graph) {
        const int rc = replay_steps(
            p, a->T, f->cur, st, [&](int c, hipStream_t cs) { full_step_b(p, f, c, eo, every, &w, cs); }, &s);
        if (rc) return rc;
    }
    for (; s < a->T; ++s) {
        full_step_b(p, f, f->cur, eo, every, &w, st);
        f->cur = 1 - f->cur;
    }
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

extern "C" int rbffd_set_field_hv(rbffd_plan* p, const double* c_dev, void* stream) {
    if (!p) return RBFFD_EINVAL;
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    if (p->K < 2 || !p->gk) return set_err(p, RBFFD_ENOTSUP, "per-field hyperviscosity needs a K-field batch");
    if (p->p.hv_alpha < 1) return set_err(p, RBFFD_ENOTSUP, "the plan has no hyperviscosity (hv_alpha = 0)");
    return fill_field_gamma(p, c_dev, (hipStream_t)stream);
}

// K-section search of the lower edge of the accepted interval of c (Section
// 5.1 parameter sweep, Section 6 energy band): every round runs the K fields
// from the same state, field k with c_k = c_lo (c_hi / c_lo)^(k / (K - 1)),
// and keeps the bracket [c_{k*-1}, c_{k*}] around the smallest accepted c.
extern "C" int rbffd_hv_scan(rbffd_plan* p, rbffd_fields* f, rbffd_hv_scan_args* a, void* ws, void* stream) {
    if (!p || !a) return RBFFD_EINVAL;
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    if (p->K < 3 || !p->gk) return set_err(p, RBFFD_ENOTSUP, "the scan needs a K-field batch with K >= 3");
    if (p->p.hv_alpha < 1) return set_err(p, RBFFD_ENOTSUP, "the plan has no hyperviscosity (hv_alpha = 0)");
    if (!f || !ws || !a->E0 || !a->H0 || !a->c_dev || !a->energy_dev)
        return set_err(p, RBFFD_EINVAL, "scan needs fields, workspace, initial state and device buffers");
    if (!(a->c_lo > 0 && a->c_hi > a->c_lo && std::isfinite(a->c_hi)))
        return set_err(p, RBFFD_EINVAL, "need 0 < c_lo < c_hi");
    if (a->rounds < 1 || a->T < 1 || a->energy_every < 1) return set_err(p, RBFFD_EINVAL, "rounds, T, energy_every >= 1");
    if (!(a->u_lo < a->u_hi)) return set_err(p, RBFFD_EINVAL, "need u_lo < u_hi");
    for (int b = 0; b < 2; ++b)
        if (!f->E[b] || !f->H[b]) return set_err(p, RBFFD_EINVAL, "null field buffer");
    if (f->cur != 0 && f->cur != 1) return set_err(p, RBFFD_EINVAL, "fields.cur must be 0 or 1");
    hipStream_t st = (hipStream_t)stream;
    const int K = p->K;
    const int ne = (a->T - 1) / a->energy_every + 1;
    std::vector<double> cs(K), en((size_t)ne * K);
    double lo = a->c_lo, hi = a->c_hi, best = 0.0;
    int status = 0, r = 0;
    for (; r < a->rounds; ++r) {
        for (int k = 0; k < K; ++k) cs[k] = lo * std::pow(hi / lo, (double)k / (double)(K - 1));
        HIPCHK(p, hipMemcpyAsync(a->c_dev, cs.data(), K * sizeof(double), hipMemcpyHostToDevice, st));
        int rc = fill_field_gamma(p, a->c_dev, st);
        if (rc) return rc;
        const int64_t re = p->E.N * p->FE, rh = p->E.N * p->FH;
        hipLaunchKernelGGL(k_broadcast, dim3((unsigned)cdiv(re * K, 256)), dim3(256), 0, st, (const float*)a->E0,
                           (float*)f->E[f->cur], re, K);
        hipLaunchKernelGGL(k_broadcast, dim3((unsigned)cdiv(rh * K, 256)), dim3(256), 0, st, (const float*)a->H0,
                           (float*)f->H[f->cur], rh, K);
        HIPCHK(p, hipGetLastError());
        rbffd_run_args ra{};
        ra.T = a->T;
        ra.energy_every = a->energy_every;
        ra.energy_out = a->energy_dev;
        ra.use_graph = 1;
        if ((rc = batched_run(p, f, &ra, ws, st))) return rc;
        HIPCHK(p, hipMemcpyAsync(en.data(), a->energy_dev, en.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(p, hipStreamSynchronize(st));
        int first = -1;
        for (int k = 0; k < K; ++k) {
            double umin = INFINITY, umax = -INFINITY;
            bool ok = true;
            for (int s = 0; s < ne; ++s) {
                const double u = en[(size_t)s * K + k] / en[k];
                if (!std::isfinite(u)) {
                    ok = false;
                    umax = INFINITY;
                    continue;
                }
                umin = std::min(umin, u);
                umax = std::max(umax, u);
                if (u < a->u_lo || u > a->u_hi) ok = false;
            }
            if (a->c_host) a->c_host[(size_t)r * K + k] = cs[k];
            if (a->umin_host) a->umin_host[(size_t)r * K + k] = umin;
            if (a->umax_host) a->umax_host[(size_t)r * K + k] = umax;
            if (a->ok_host) a->ok_host[(size_t)r * K + k] = ok ? 1 : 0;
            if (ok && first < 0) first = k;
        }
        if (first < 0) {
            if (best == 0.0) status = 2;
            ++r;
            break;
        }
        best = cs[first];
        if (first == 0) {
            status = 1;
            ++r;
            break;
        }
        lo = cs[first - 1];
        hi = cs[first];
    }
    a->rounds_done = r;
    a->status = status;
    a->c_best = best;
    a->bracket[0] = lo;
    a->bracket[1] = hi;
    // later runs use the plan's c again
    int rc = fill_field_gamma(p, nullptr, st);
    if (rc) return rc;
    HIPCHK(p, hipStreamSynchronize(st));
    return RBFFD_OK;
}
