// The hot path: one fused kernel per half step of the stabilised leapfrog
// (Kolar-Pozun & Kosec, arXiv 2508.18205, Section 5, eq. 19; 3D with the full
// discrete curl), plus the step loop (sources, receivers, energy of eq. 20,
// checkpoints, HIP-graph replay) and the FP64 reductions.
//
// Per node i the H update is
//   H_i <- H_i + a (-curl_D E)_i + a gamma (D^hv H)_i          a = dt / mu0
// and the E update
//   E_i <- mask_i [ E_i + kappa_i ((curl_D H_new)_i + gamma (D^hv E)_i) ]
// with kappa_i = dt / (eps0 eps_r,i) and mask = the PEC projector.  All
// operators are applied in difference form sum_s w_s (f_s - f_ref) with the
// reference slot left out (the weights sum to zero), which keeps the FP32
// sums free of the cancellation of sum_s w_s f_s.
//
// One wavefront owns one 64-node tile; its lanes stream the tile's packed
// indices and weights with 16-byte loads and gather field values through the
// L2 (nodes are Morton ordered, tiles are mapped XCD-contiguously).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.h"
#include "fields.h"
#include "wpack.h"

namespace {

template <typename TS, typename TW>
struct SA {
    const TS* E;          // E^n
    const TS* H;          // H update: H^n ; E update: H^{n+1}
    TS* out;              // H^{n+1} or E^{n+1}
    const int4* idx;      // collocated: union chunks ; two-set: curl chunks
    const int4* idx_h;    // two-set: hv chunks
    const int32_t* pref;  // two-set: curl reference node
    const TW* wc;
    const TW* wh;
    int64_t N, tiles;
    int C4, V4, S4;
    int xcd;
    double a;             // H update: dt / mu0 ; E update: dt / eps0
    double g;             // gamma
    double dt, eps0;
    const void* eps_r;    // per-node eps_r (double for FP64 fields, else float) or null
    const uint8_t* emask;
    const double* wnrm;   // [N][dim] unit wall normals (TEz and 3D curved walls; emask bit 3)
    // TEz: the 2D kernels with the fields' roles exchanged.  te = 1: the
    // vector kernel updates (Ex, Ey) from Hz with factor -kappa_i and the wall
    // mask; nomask = 1: the scalar kernel updates Hz (no wall mask)
    int te, nomask;
    // LDS staging
    const uint4* lidx;    // [tiles][Q8][64] x 8 u16 halo positions
    const int32_t* hpool;
    const int32_t* hoff;
    int Q8, hmax;
};

// PEC on the in-plane E of the TEz polarisation: bit 0 / 1 of the mask keeps
// Ex / Ey (walls normal to an axis); bit 3 marks a curved-wall node with unit
// normal n = wn[i], where only the normal component survives: E <- (E . n) n
// The same for the 3D E: bits 0..2 keep Ex, Ey, Ez (faces normal to an axis),
// bit 3 projects on the unit normal wn[i] (curved wall)
template <typename TC>
__device__ __forceinline__ void wall3(uint8_t m, const double* wn, int64_t i, TC& x, TC& y, TC& z) {
    if (m & 8) {
        const TC nx = (TC)wn[3 * i], ny = (TC)wn[3 * i + 1], nz = (TC)wn[3 * i + 2];
        const TC en = x * nx + y * ny + z * nz;
        x = en * nx;
        y = en * ny;
        z = en * nz;
    } else {
        x = (m & 1) ? x : (TC)0;
        y = (m & 2) ? y : (TC)0;
        z = (m & 4) ? z : (TC)0;
    }
}

template <typename TC>
__device__ __forceinline__ void te_wall(uint8_t m, const double* wn, int64_t i, TC& x, TC& y) {
    if (m & 8) {
        const TC nx = (TC)wn[2 * i], ny = (TC)wn[2 * i + 1];
        const TC en = x * nx + y * ny;
        x = en * nx;
        y = en * ny;
    } else {
        x = (m & 1) ? x : (TC)0;
        y = (m & 2) ? y : (TC)0;
    }
}

template <typename TS, typename TW>
__device__ __forceinline__ int64_t tile_of(const SA<TS, TW>& a) {
    const int wpb = blockDim.x >> 6;
    const int blk = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    return (int64_t)blk * wpb + (threadIdx.x >> 6);
}

template <typename TS, typename TW>
__device__ __forceinline__ typename Store<TS>::C kappa_of(const SA<TS, TW>& a, int64_t i) {
    using TC = typename Store<TS>::C;
    if (!a.eps_r) return (TC)a.a;
    if (sizeof(TC) == 8) return (TC)(a.dt / (a.eps0 * ((const double*)a.eps_r)[i]));
    return (TC)(a.dt / (a.eps0 * (double)((const float*)a.eps_r)[i]));
}

// ---- 2D TMz, collocated ----------------------------------------------------
template <typename TS, typename TW>
__global__ __launch_bounds__(512) void k_h2(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    using WV = typename WF<TW>::V;
    const int64_t tile = tile_of(a);
    if (tile >= a.tiles) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    const TC e0 = S::ld1(a.E, ic);
    TC hx0, hy0;
    S::ld2(a.H, ic, hx0, hy0);
    TC dx = 0, dy = 0, vx = 0, vy = 0;
    const int4* pi = a.idx + tile * a.S4 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 2 * WF<TW>::CH + lane * WF<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * WF<TW>::CH + lane * WF<TW>::LS;
    const int qb = min(a.C4, a.V4);
    int q = 0;
    for (; q < qb; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        WV wx[4], wy[4], wh[4];
        WF<TW>::ldp(pc + (q * 2 + 0) * WF<TW>::CH, wx);
        WF<TW>::ldp(pc + (q * 2 + 1) * WF<TW>::CH, wy);
        WF<TW>::ldp(ph + q * WF<TW>::CH, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int jj = idx4(j, u);
            const TC de = S::ld1(a.E, jj) - e0;
            dx += (TC)wx[u] * de;
            dy += (TC)wy[u] * de;
            TC hx, hy;
            S::ld2(a.H, jj, hx, hy);
            vx += (TC)wh[u] * (hx - hx0);
            vy += (TC)wh[u] * (hy - hy0);
        }
    }
    for (; q < a.C4; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        WV wx[4], wy[4];
        WF<TW>::ldp(pc + (q * 2 + 0) * WF<TW>::CH, wx);
        WF<TW>::ldp(pc + (q * 2 + 1) * WF<TW>::CH, wy);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const TC de = S::ld1(a.E, idx4(j, u)) - e0;
            dx += (TC)wx[u] * de;
            dy += (TC)wy[u] * de;
        }
    }
    for (; q < a.V4; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        WV wh[4];
        WF<TW>::ldp(ph + q * WF<TW>::CH, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC hx, hy;
            S::ld2(a.H, idx4(j, u), hx, hy);
            vx += (TC)wh[u] * (hx - hx0);
            vy += (TC)wh[u] * (hy - hy0);
        }
    }
    if (i < a.N) {
        const TC G = (TC)a.g;
        if (!a.te) {
            const TC A = (TC)a.a;
            S::st2(a.out, i, hx0 + A * (-dy + G * vx), hy0 + A * (dx + G * vy));
        } else {
            // TEz (Ex, Ey) <- E + kappa (D^dy Hz + gamma HV, -D^dx Hz + gamma HV),
            // written as E - kappa (-D^dy Hz - gamma HV, D^dx Hz - gamma HV) with
            // the host's gamma negated; then the wall mask
            const TC A = -kappa_of(a, i);
            TC ex = hx0 + A * (-dy + G * vx), ey = hy0 + A * (dx + G * vy);
            te_wall(a.emask[i], a.wnrm, i, ex, ey);
            S::st2(a.out, i, ex, ey);
        }
    }
}

template <typename TS, typename TW>
__global__ __launch_bounds__(512) void k_e2(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    using WV = typename WF<TW>::V;
    const int64_t tile = tile_of(a);
    if (tile >= a.tiles) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    const TC e0 = S::ld1(a.E, ic);
    TC hx0, hy0;
    S::ld2(a.H, ic, hx0, hy0);
    TC cu = 0, ve = 0;
    const int4* pi = a.idx + tile * a.S4 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 2 * WF<TW>::CH + lane * WF<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * WF<TW>::CH + lane * WF<TW>::LS;
    const int qb = min(a.C4, a.V4);
    int q = 0;
    for (; q < qb; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        WV wx[4], wy[4], wh[4];
        WF<TW>::ldp(pc + (q * 2 + 0) * WF<TW>::CH, wx);
        WF<TW>::ldp(pc + (q * 2 + 1) * WF<TW>::CH, wy);
        WF<TW>::ldp(ph + q * WF<TW>::CH, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int jj = idx4(j, u);
            TC hx, hy;
            S::ld2(a.H, jj, hx, hy);
            cu += (TC)wx[u] * (hy - hy0) - (TC)wy[u] * (hx - hx0);
            ve += (TC)wh[u] * (S::ld1(a.E, jj) - e0);
        }
    }
    for (; q < a.C4; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        WV wx[4], wy[4];
        WF<TW>::ldp(pc + (q * 2 + 0) * WF<TW>::CH, wx);
        WF<TW>::ldp(pc + (q * 2 + 1) * WF<TW>::CH, wy);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC hx, hy;
            S::ld2(a.H, idx4(j, u), hx, hy);
            cu += (TC)wx[u] * (hy - hy0) - (TC)wy[u] * (hx - hx0);
        }
    }
    for (; q < a.V4; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        WV wh[4];
        WF<TW>::ldp(ph + q * WF<TW>::CH, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) ve += (TC)wh[u] * (S::ld1(a.E, idx4(j, u)) - e0);
    }
    if (i < a.N) {
        const TC k = kappa_of(a, i);
        const TC v = (a.nomask || (a.emask[i] & 1)) ? e0 + k * (cu + (TC)a.g * ve) : (TC)0;
        S::st1(a.out, i, v);
    }
}

// ---- 2D TMz, two node sets ---------------------------------------------------
// H update: curl of E from the E set (reference = nearest E node), HV of H on
// the H set.  E update: curl of H from the H set, HV of E on the E set.
template <typename TS, typename TW>
__global__ __launch_bounds__(512) void k_h2x(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    const int64_t tile = tile_of(a);
    if (tile >= a.tiles) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    const TC e0 = S::ld1(a.E, a.pref[ic]);
    TC hx0, hy0;
    S::ld2(a.H, ic, hx0, hy0);
    TC dx = 0, dy = 0, vx = 0, vy = 0;
    const int4* pi = a.idx + tile * a.C4 * RBFFD_TILE + lane;
    const int4* pj = a.idx_h + tile * a.V4 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 2 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    for (int q = 0; q < a.C4; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        TW wx[4], wy[4];
        ldw4p(pc + (q * 2 + 0) * RBFFD_TILE * 4, wx);
        ldw4p(pc + (q * 2 + 1) * RBFFD_TILE * 4, wy);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const TC de = S::ld1(a.E, idx4(j, u)) - e0;
            dx += (TC)wx[u] * de;
            dy += (TC)wy[u] * de;
        }
    }
    for (int q = 0; q < a.V4; ++q) {
        const int4 j = pj[q * RBFFD_TILE];
        TW wh[4];
        ldw4p(ph + q * RBFFD_TILE * 4, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC hx, hy;
            S::ld2(a.H, idx4(j, u), hx, hy);
            vx += (TC)wh[u] * (hx - hx0);
            vy += (TC)wh[u] * (hy - hy0);
        }
    }
    if (i < a.N) {
        const TC G = (TC)a.g;
        if (!a.te) {
            const TC A = (TC)a.a;
            S::st2(a.out, i, hx0 + A * (-dy + G * vx), hy0 + A * (dx + G * vy));
        } else {
            // TEz (Ex, Ey) <- E + kappa (D^dy Hz + gamma HV, -D^dx Hz + gamma HV),
            // written as E - kappa (-D^dy Hz - gamma HV, D^dx Hz - gamma HV) with
            // the host's gamma negated; then the wall mask
            const TC A = -kappa_of(a, i);
            TC ex = hx0 + A * (-dy + G * vx), ey = hy0 + A * (dx + G * vy);
            te_wall(a.emask[i], a.wnrm, i, ex, ey);
            S::st2(a.out, i, ex, ey);
        }
    }
}

template <typename TS, typename TW>
__global__ __launch_bounds__(512) void k_e2x(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    const int64_t tile = tile_of(a);
    if (tile >= a.tiles) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    const TC e0 = S::ld1(a.E, ic);
    TC hx0, hy0;
    S::ld2(a.H, a.pref[ic], hx0, hy0);
    TC cu = 0, ve = 0;
    const int4* pi = a.idx + tile * a.C4 * RBFFD_TILE + lane;
    const int4* pj = a.idx_h + tile * a.V4 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 2 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    for (int q = 0; q < a.C4; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        TW wx[4], wy[4];
        ldw4p(pc + (q * 2 + 0) * RBFFD_TILE * 4, wx);
        ldw4p(pc + (q * 2 + 1) * RBFFD_TILE * 4, wy);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC hx, hy;
            S::ld2(a.H, idx4(j, u), hx, hy);
            cu += (TC)wx[u] * (hy - hy0) - (TC)wy[u] * (hx - hx0);
        }
    }
    for (int q = 0; q < a.V4; ++q) {
        const int4 j = pj[q * RBFFD_TILE];
        TW wh[4];
        ldw4p(ph + q * RBFFD_TILE * 4, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) ve += (TC)wh[u] * (S::ld1(a.E, idx4(j, u)) - e0);
    }
    if (i < a.N) {
        const TC k = kappa_of(a, i);
        const TC v = (a.nomask || (a.emask[i] & 1)) ? e0 + k * (cu + (TC)a.g * ve) : (TC)0;
        S::st1(a.out, i, v);
    }
}

// ---- 2D, two node sets, small node sets ---------------------------------------
// As k_h2x / k_e2x with one 64-node tile per workgroup: its four wavefronts
// each sum every fourth curl chunk and every fourth hyperviscosity chunk, and
// the partial sums meet in LDS in a fixed order (the small-set scheme of
// k_h2s / k_e2s below, for the staggered variant).
template <typename TS, typename TW>
__global__ __launch_bounds__(256) void k_h2xs(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    __shared__ TC part[3][4][RBFFD_TILE];
    const int64_t tile = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    const TC e0 = S::ld1(a.E, a.pref[ic]);
    TC hx0, hy0;
    S::ld2(a.H, ic, hx0, hy0);
    TC dx = 0, dy = 0, vx = 0, vy = 0;
    const int4* pi = a.idx + tile * a.C4 * RBFFD_TILE + lane;
    const int4* pj = a.idx_h + tile * a.V4 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 2 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    for (int q = r; q < a.C4; q += 4) {
        const int4 j = pi[q * RBFFD_TILE];
        TW wx[4], wy[4];
        ldw4p(pc + (q * 2 + 0) * RBFFD_TILE * 4, wx);
        ldw4p(pc + (q * 2 + 1) * RBFFD_TILE * 4, wy);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const TC de = S::ld1(a.E, idx4(j, u)) - e0;
            dx += (TC)wx[u] * de;
            dy += (TC)wy[u] * de;
        }
    }
    for (int q = r; q < a.V4; q += 4) {
        const int4 j = pj[q * RBFFD_TILE];
        TW wh[4];
        ldw4p(ph + q * RBFFD_TILE * 4, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC hx, hy;
            S::ld2(a.H, idx4(j, u), hx, hy);
            vx += (TC)wh[u] * (hx - hx0);
            vy += (TC)wh[u] * (hy - hy0);
        }
    }
    if (r > 0) {
        part[r - 1][0][lane] = dx;
        part[r - 1][1][lane] = dy;
        part[r - 1][2][lane] = vx;
        part[r - 1][3][lane] = vy;
    }
    __syncthreads();
    if (r > 0 || i >= a.N) return;
    dx = ((dx + part[0][0][lane]) + part[1][0][lane]) + part[2][0][lane];
    dy = ((dy + part[0][1][lane]) + part[1][1][lane]) + part[2][1][lane];
    vx = ((vx + part[0][2][lane]) + part[1][2][lane]) + part[2][2][lane];
    vy = ((vy + part[0][3][lane]) + part[1][3][lane]) + part[2][3][lane];
    const TC G = (TC)a.g;
    if (!a.te) {
        const TC A = (TC)a.a;
        S::st2(a.out, i, hx0 + A * (-dy + G * vx), hy0 + A * (dx + G * vy));
    } else {
        const TC A = -kappa_of(a, i);
        TC ex = hx0 + A * (-dy + G * vx), ey = hy0 + A * (dx + G * vy);
        te_wall(a.emask[i], a.wnrm, i, ex, ey);
        S::st2(a.out, i, ex, ey);
    }
}

template <typename TS, typename TW>
__global__ __launch_bounds__(256) void k_e2xs(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    __shared__ TC part[3][2][RBFFD_TILE];
    const int64_t tile = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    const TC e0 = S::ld1(a.E, ic);
    TC hx0, hy0;
    S::ld2(a.H, a.pref[ic], hx0, hy0);
    TC cu = 0, ve = 0;
    const int4* pi = a.idx + tile * a.C4 * RBFFD_TILE + lane;
    const int4* pj = a.idx_h + tile * a.V4 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 2 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    for (int q = r; q < a.C4; q += 4) {
        const int4 j = pi[q * RBFFD_TILE];
        TW wx[4], wy[4];
        ldw4p(pc + (q * 2 + 0) * RBFFD_TILE * 4, wx);
        ldw4p(pc + (q * 2 + 1) * RBFFD_TILE * 4, wy);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC hx, hy;
            S::ld2(a.H, idx4(j, u), hx, hy);
            cu += (TC)wx[u] * (hy - hy0) - (TC)wy[u] * (hx - hx0);
        }
    }
    for (int q = r; q < a.V4; q += 4) {
        const int4 j = pj[q * RBFFD_TILE];
        TW wh[4];
        ldw4p(ph + q * RBFFD_TILE * 4, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) ve += (TC)wh[u] * (S::ld1(a.E, idx4(j, u)) - e0);
    }
    if (r > 0) {
        part[r - 1][0][lane] = cu;
        part[r - 1][1][lane] = ve;
    }
    __syncthreads();
    if (r > 0 || i >= a.N) return;
    cu = ((cu + part[0][0][lane]) + part[1][0][lane]) + part[2][0][lane];
    ve = ((ve + part[0][1][lane]) + part[1][1][lane]) + part[2][1][lane];
    const TC k = kappa_of(a, i);
    const TC v = (a.nomask || (a.emask[i] & 1)) ? e0 + k * (cu + (TC)a.g * ve) : (TC)0;
    S::st1(a.out, i, v);
}

// ---- 2D, collocated, small node sets ----------------------------------------
// One 64-node tile per workgroup; its four wavefronts each sum every fourth
// slot chunk of the tile's nodes (every load is still one contiguous run per
// wavefront) and the partial sums meet in LDS in a fixed order.  The chain
// of dependent loads per node is four times shorter, for launches too small
// to fill the chip.  Same terms as k_h2 / k_e2; only the order of the partial
// sums differs.
template <typename TS, typename TW>
__global__ __launch_bounds__(256) void k_h2s(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    using WV = typename WF<TW>::V;
    __shared__ TC part[3][4][RBFFD_TILE];
    const int64_t tile = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    const TC e0 = S::ld1(a.E, ic);
    TC hx0, hy0;
    S::ld2(a.H, ic, hx0, hy0);
    TC dx = 0, dy = 0, vx = 0, vy = 0;
    const int4* pi = a.idx + tile * a.S4 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 2 * WF<TW>::CH + lane * WF<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * WF<TW>::CH + lane * WF<TW>::LS;
    const int qm = max(a.C4, a.V4);
    for (int q = r; q < qm; q += 4) {
        const int4 j = pi[q * RBFFD_TILE];
        if (q < a.C4) {
            WV wx[4], wy[4];
            WF<TW>::ldp(pc + (q * 2 + 0) * WF<TW>::CH, wx);
            WF<TW>::ldp(pc + (q * 2 + 1) * WF<TW>::CH, wy);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const TC de = S::ld1(a.E, idx4(j, u)) - e0;
                dx += (TC)wx[u] * de;
                dy += (TC)wy[u] * de;
            }
        }
        if (q < a.V4) {
            WV wh[4];
            WF<TW>::ldp(ph + q * WF<TW>::CH, wh);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                TC hx, hy;
                S::ld2(a.H, idx4(j, u), hx, hy);
                vx += (TC)wh[u] * (hx - hx0);
                vy += (TC)wh[u] * (hy - hy0);
            }
        }
    }
    if (r > 0) {
        part[r - 1][0][lane] = dx;
        part[r - 1][1][lane] = dy;
        part[r - 1][2][lane] = vx;
        part[r - 1][3][lane] = vy;
    }
    __syncthreads();
    if (r > 0 || i >= a.N) return;
    dx = ((dx + part[0][0][lane]) + part[1][0][lane]) + part[2][0][lane];
    dy = ((dy + part[0][1][lane]) + part[1][1][lane]) + part[2][1][lane];
    vx = ((vx + part[0][2][lane]) + part[1][2][lane]) + part[2][2][lane];
    vy = ((vy + part[0][3][lane]) + part[1][3][lane]) + part[2][3][lane];
    const TC G = (TC)a.g;
    if (!a.te) {
        const TC A = (TC)a.a;
        S::st2(a.out, i, hx0 + A * (-dy + G * vx), hy0 + A * (dx + G * vy));
    } else {
        const TC A = -kappa_of(a, i);
        TC ex = hx0 + A * (-dy + G * vx), ey = hy0 + A * (dx + G * vy);
        te_wall(a.emask[i], a.wnrm, i, ex, ey);
        S::st2(a.out, i, ex, ey);
    }
}

template <typename TS, typename TW>
__global__ __launch_bounds__(256) void k_e2s(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    using WV = typename WF<TW>::V;
    __shared__ TC part[3][2][RBFFD_TILE];
    const int64_t tile = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    const TC e0 = S::ld1(a.E, ic);
    TC hx0, hy0;
    S::ld2(a.H, ic, hx0, hy0);
    TC cu = 0, ve = 0;
    const int4* pi = a.idx + tile * a.S4 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 2 * WF<TW>::CH + lane * WF<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * WF<TW>::CH + lane * WF<TW>::LS;
    const int qm = max(a.C4, a.V4);
    for (int q = r; q < qm; q += 4) {
        const int4 j = pi[q * RBFFD_TILE];
        if (q < a.C4) {
            WV wx[4], wy[4];
            WF<TW>::ldp(pc + (q * 2 + 0) * WF<TW>::CH, wx);
            WF<TW>::ldp(pc + (q * 2 + 1) * WF<TW>::CH, wy);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                TC hx, hy;
                S::ld2(a.H, idx4(j, u), hx, hy);
                cu += (TC)wx[u] * (hy - hy0) - (TC)wy[u] * (hx - hx0);
            }
        }
        if (q < a.V4) {
            WV wh[4];
            WF<TW>::ldp(ph + q * WF<TW>::CH, wh);
#pragma unroll
            for (int u = 0; u < 4; ++u) ve += (TC)wh[u] * (S::ld1(a.E, idx4(j, u)) - e0);
        }
    }
    if (r > 0) {
        part[r - 1][0][lane] = cu;
        part[r - 1][1][lane] = ve;
    }
    __syncthreads();
    if (r > 0 || i >= a.N) return;
    cu = ((cu + part[0][0][lane]) + part[1][0][lane]) + part[2][0][lane];
    ve = ((ve + part[0][1][lane]) + part[1][1][lane]) + part[2][1][lane];
    const TC k = kappa_of(a, i);
    const TC v = (a.nomask || (a.emask[i] & 1)) ? e0 + k * (cu + (TC)a.g * ve) : (TC)0;
    S::st1(a.out, i, v);
}

// ---- 3D, collocated: E and H stored as (x, y, z, pad) -------------------------
template <typename TS, typename TW>
__global__ __launch_bounds__(512) void k_h3(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    const int64_t tile = tile_of(a);
    if (tile >= a.tiles) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    TC ex0, ey0, ez0, hx0, hy0, hz0;
    S::ld3(a.E, ic, ex0, ey0, ez0);
    S::ld3(a.H, ic, hx0, hy0, hz0);
    // d_a E_c accumulators for the curl
    TC xEy = 0, xEz = 0, yEx = 0, yEz = 0, zEx = 0, zEy = 0, vx = 0, vy = 0, vz = 0;
    const int4* pi = a.idx + tile * a.S4 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 3 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const int qb = min(a.C4, a.V4);
    int q = 0;
    for (; q < qb; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        TW wx[4], wy[4], wz[4], wh[4];
        ldw4p(pc + (q * 3 + 0) * RBFFD_TILE * 4, wx);
        ldw4p(pc + (q * 3 + 1) * RBFFD_TILE * 4, wy);
        ldw4p(pc + (q * 3 + 2) * RBFFD_TILE * 4, wz);
        ldw4p(ph + q * RBFFD_TILE * 4, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int jj = idx4(j, u);
            TC ex, ey, ez, hx, hy, hz;
            S::ld3(a.E, jj, ex, ey, ez);
            S::ld3(a.H, jj, hx, hy, hz);
            ex -= ex0; ey -= ey0; ez -= ez0;
            xEy += (TC)wx[u] * ey; xEz += (TC)wx[u] * ez;
            yEx += (TC)wy[u] * ex; yEz += (TC)wy[u] * ez;
            zEx += (TC)wz[u] * ex; zEy += (TC)wz[u] * ey;
            vx += (TC)wh[u] * (hx - hx0);
            vy += (TC)wh[u] * (hy - hy0);
            vz += (TC)wh[u] * (hz - hz0);
        }
    }
    for (; q < a.C4; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        TW wx[4], wy[4], wz[4];
        ldw4p(pc + (q * 3 + 0) * RBFFD_TILE * 4, wx);
        ldw4p(pc + (q * 3 + 1) * RBFFD_TILE * 4, wy);
        ldw4p(pc + (q * 3 + 2) * RBFFD_TILE * 4, wz);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC ex, ey, ez;
            S::ld3(a.E, idx4(j, u), ex, ey, ez);
            ex -= ex0; ey -= ey0; ez -= ez0;
            xEy += (TC)wx[u] * ey; xEz += (TC)wx[u] * ez;
            yEx += (TC)wy[u] * ex; yEz += (TC)wy[u] * ez;
            zEx += (TC)wz[u] * ex; zEy += (TC)wz[u] * ey;
        }
    }
    for (; q < a.V4; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        TW wh[4];
        ldw4p(ph + q * RBFFD_TILE * 4, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC hx, hy, hz;
            S::ld3(a.H, idx4(j, u), hx, hy, hz);
            vx += (TC)wh[u] * (hx - hx0);
            vy += (TC)wh[u] * (hy - hy0);
            vz += (TC)wh[u] * (hz - hz0);
        }
    }
    if (i < a.N) {
        const TC A = (TC)a.a, G = (TC)a.g;
        // H <- H - a (curl E - gamma D^hv H)
        S::st3(a.out, i, hx0 - A * ((yEz - zEy) - G * vx), hy0 - A * ((zEx - xEz) - G * vy),
               hz0 - A * ((xEy - yEx) - G * vz));
    }
}

template <typename TS, typename TW>
__global__ __launch_bounds__(512) void k_e3(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    const int64_t tile = tile_of(a);
    if (tile >= a.tiles) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    TC ex0, ey0, ez0, hx0, hy0, hz0;
    S::ld3(a.E, ic, ex0, ey0, ez0);
    S::ld3(a.H, ic, hx0, hy0, hz0);
    TC xHy = 0, xHz = 0, yHx = 0, yHz = 0, zHx = 0, zHy = 0, vx = 0, vy = 0, vz = 0;
    const int4* pi = a.idx + tile * a.S4 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 3 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const int qb = min(a.C4, a.V4);
    int q = 0;
    for (; q < qb; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        TW wx[4], wy[4], wz[4], wh[4];
        ldw4p(pc + (q * 3 + 0) * RBFFD_TILE * 4, wx);
        ldw4p(pc + (q * 3 + 1) * RBFFD_TILE * 4, wy);
        ldw4p(pc + (q * 3 + 2) * RBFFD_TILE * 4, wz);
        ldw4p(ph + q * RBFFD_TILE * 4, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int jj = idx4(j, u);
            TC ex, ey, ez, hx, hy, hz;
            S::ld3(a.H, jj, hx, hy, hz);
            S::ld3(a.E, jj, ex, ey, ez);
            hx -= hx0; hy -= hy0; hz -= hz0;
            xHy += (TC)wx[u] * hy; xHz += (TC)wx[u] * hz;
            yHx += (TC)wy[u] * hx; yHz += (TC)wy[u] * hz;
            zHx += (TC)wz[u] * hx; zHy += (TC)wz[u] * hy;
            vx += (TC)wh[u] * (ex - ex0);
            vy += (TC)wh[u] * (ey - ey0);
            vz += (TC)wh[u] * (ez - ez0);
        }
    }
    for (; q < a.C4; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        TW wx[4], wy[4], wz[4];
        ldw4p(pc + (q * 3 + 0) * RBFFD_TILE * 4, wx);
        ldw4p(pc + (q * 3 + 1) * RBFFD_TILE * 4, wy);
        ldw4p(pc + (q * 3 + 2) * RBFFD_TILE * 4, wz);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC hx, hy, hz;
            S::ld3(a.H, idx4(j, u), hx, hy, hz);
            hx -= hx0; hy -= hy0; hz -= hz0;
            xHy += (TC)wx[u] * hy; xHz += (TC)wx[u] * hz;
            yHx += (TC)wy[u] * hx; yHz += (TC)wy[u] * hz;
            zHx += (TC)wz[u] * hx; zHy += (TC)wz[u] * hy;
        }
    }
    for (; q < a.V4; ++q) {
        const int4 j = pi[q * RBFFD_TILE];
        TW wh[4];
        ldw4p(ph + q * RBFFD_TILE * 4, wh);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC ex, ey, ez;
            S::ld3(a.E, idx4(j, u), ex, ey, ez);
            vx += (TC)wh[u] * (ex - ex0);
            vy += (TC)wh[u] * (ey - ey0);
            vz += (TC)wh[u] * (ez - ez0);
        }
    }
    if (i < a.N) {
        const TC k = kappa_of(a, i), G = (TC)a.g;
        TC nx = ex0 + k * ((yHz - zHy) + G * vx);
        TC ny = ey0 + k * ((zHx - xHz) + G * vy);
        TC nz = ez0 + k * ((xHy - yHx) + G * vz);
        wall3(a.emask[i], a.wnrm, i, nx, ny, nz);
        S::st3(a.out, i, nx, ny, nz);
    }
}

// ---- LDS-staged variants ------------------------------------------------------
// A workgroup owns 256 consecutive nodes in 2D, in 3D 1024 with FP32 weights
// and 512 with FP64 (4, 16 or 8 wavefront tiles).  It first copies
// the field values of every node its stencils touch (the sorted halo list)
// into LDS with one coalesced pass, then each node sums over its slots with
// 16-bit halo positions (8 per 16-byte load) instead of 32-bit global indices
// and global gathers.  Same arithmetic and summation order as the global
// variants.
__device__ __forceinline__ int pos4(const uint4& v, int half, int u) {
    const uint32_t w = half ? (u < 2 ? v.z : v.w) : (u < 2 ? v.x : v.y);
    return (int)((u & 1) ? (w >> 16) : (w & 0xFFFFu));
}

template <typename TW>
__device__ __forceinline__ void copy4(TW (&d)[4], const TW (&s)[4]) {
    d[0] = s[0];
    d[1] = s[1];
    d[2] = s[2];
    d[3] = s[3];
}
// weights of chunk q of a 2D block (left unchanged past the chunk counts)
template <typename TW, typename WV = typename WF<TW>::V>
__device__ __forceinline__ void load2(const TW* pc, const TW* ph, int q, int C4, int V4, WV (&x)[4], WV (&y)[4],
                                      WV (&h)[4]) {
    if (q < C4) {
        WF<TW>::ld(pc + (q * 2 + 0) * WF<TW>::CH, x);
        WF<TW>::ld(pc + (q * 2 + 1) * WF<TW>::CH, y);
    }
    if (q < V4) WF<TW>::ld(ph + q * WF<TW>::CH, h);
}

// weights of chunk q of a 3D block (left unchanged past the chunk counts)
template <typename TW>
__device__ __forceinline__ void load3(const TW* pc, const TW* ph, int q, int C4, int V4, TW (&x)[4], TW (&y)[4],
                                      TW (&z)[4], TW (&h)[4]) {
    if (q < C4) {
        ldw4(pc + (q * 3 + 0) * RBFFD_TILE * 4, x);
        ldw4(pc + (q * 3 + 1) * RBFFD_TILE * 4, y);
        ldw4(pc + (q * 3 + 2) * RBFFD_TILE * 4, z);
    }
    if (q < V4) ldw4(ph + q * RBFFD_TILE * 4, h);
}

// 3-vector LDS entries, packed (12 B in FP32) so that more workgroups fit
template <typename TC>
__device__ __forceinline__ void st_lds3(TC* p, const TC (&v)[3]) {
    p[0] = v[0];
    p[1] = v[1];
    p[2] = v[2];
}
template <typename TC>
__device__ __forceinline__ void ld_lds3(const TC* p, TC (&v)[3]) {
    v[0] = p[0];
    v[1] = p[1];
    v[2] = p[2];
}

// one 16-byte (FP32) or two 16-byte (FP64) LDS accesses per 3-vector entry
__device__ __forceinline__ void st_lds4(float* p, const float (&v)[3]) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], 0.0f);
}
__device__ __forceinline__ void st_lds4(double* p, const double (&v)[3]) {
    reinterpret_cast<double2*>(p)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2*>(p)[1] = make_double2(v[2], 0.0);
}
__device__ __forceinline__ void ld_lds4(const float* p, float (&v)[3]) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
}
__device__ __forceinline__ void ld_lds4(const double* p, double (&v)[3]) {
    const double2 a = reinterpret_cast<const double2*>(p)[0];
    const double2 b = reinterpret_cast<const double2*>(p)[1];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
}

__device__ __forceinline__ void ld_lds2(const float* p, float& x, float& y) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    x = t.x;
    y = t.y;
}
__device__ __forceinline__ void ld_lds2(const double* p, double& x, double& y) {
    const double2 t = *reinterpret_cast<const double2*>(p);
    x = t.x;
    y = t.y;
}
__device__ __forceinline__ void st_lds2(float* p, float x, float y) { *reinterpret_cast<float2*>(p) = make_float2(x, y); }
__device__ __forceinline__ void st_lds2(double* p, double x, double y) {
    *reinterpret_cast<double2*>(p) = make_double2(x, y);
}

template <typename TC>
__device__ __forceinline__ TC* lds_base() {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    return reinterpret_cast<TC*>(smem_raw);
}

// Halo staging with several loads in flight per thread: each round takes up
// to SB list entries per thread, loads all their list values, then all their
// field values, then stores them (a plain loop waits for each load in turn).
// ld(j) returns the staged value of source node j, st(k, v) stores entry k.
template <int SB, typename V, typename LD, typename ST>
__device__ __forceinline__ void stage_rounds(const int32_t* list, int hc, LD ld, ST st) {
    const int nt = (int)blockDim.x, t = (int)threadIdx.x;
    for (int base = 0; base < hc; base += SB * nt) {
        int j[SB];
#pragma unroll
        for (int b = 0; b < SB; ++b) {
            const int k = base + b * nt + t;
            j[b] = k < hc ? list[k] : -1;
        }
        V v[SB];
#pragma unroll
        for (int b = 0; b < SB; ++b)
            if (j[b] >= 0) v[b] = ld(j[b]);
#pragma unroll
        for (int b = 0; b < SB; ++b)
            if (j[b] >= 0) st(base + b * nt + t, v[b]);
    }
}

template <typename TC>
struct Val3 {
    TC x, y, z;
};
template <typename TC>
struct Val6 {
    TC v[6];
};

template <typename TS, typename TW>
__global__ __launch_bounds__(256) void k_h2l(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    using WV = typename WF<TW>::V;
    TC* sE = lds_base<TC>();
    TC* sH = sE + ((a.hmax + 3) & ~3);                 // pairs (Hx, Hy)
    const int wg = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int h0 = a.hoff[wg], hc = a.hoff[wg + 1] - h0;
    stage_rounds<4, Val3<TC>>(
        a.hpool + h0, hc,
        [&](int j) {
            Val3<TC> v;
            v.x = S::ld1(a.E, j);
            S::ld2(a.H, j, v.y, v.z);
            return v;
        },
        [&](int k, const Val3<TC>& v) {
            sE[k] = v.x;
            st_lds2(sH + 2 * k, v.y, v.z);
        });
    __syncthreads();
    const int64_t tile = (int64_t)wg * (RBFFD_WGT / RBFFD_TILE) + (threadIdx.x >> 6);
    if (tile >= a.tiles) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    const TC e0 = S::ld1(a.E, ic);
    TC hx0, hy0;
    S::ld2(a.H, ic, hx0, hy0);
    TC dx = 0, dy = 0, vx = 0, vy = 0;
    const uint4* pl = a.lidx + tile * a.Q8 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 2 * WF<TW>::CH + lane * WF<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * WF<TW>::CH + lane * WF<TW>::LS;
    const int qm = max(a.C4, a.V4);
    // chunk q + 1 is loaded while chunk q is summed
    uint4 li = ldu4s(pl);
    WV nx[4] = {0, 0, 0, 0}, ny[4] = {0, 0, 0, 0}, nh[4] = {0, 0, 0, 0};
    load2(pc, ph, 0, a.C4, a.V4, nx, ny, nh);
    for (int q = 0; q < qm; ++q) {
        const uint4 lc = li;
        WV wx[4], wy[4], wh[4];
        copy4(wx, nx); copy4(wy, ny); copy4(wh, nh);
        if (q + 1 < qm) {
            if (((q + 1) & 1) == 0) li = ldu4s(pl + ((q + 1) >> 1) * RBFFD_TILE);
            load2(pc, ph, q + 1, a.C4, a.V4, nx, ny, nh);
        }
        const int hf = q & 1;
        if (q < a.C4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const TC de = sE[pos4(lc, hf, u)] - e0;
                dx += (TC)wx[u] * de;
                dy += (TC)wy[u] * de;
            }
        }
        if (q < a.V4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                TC hx, hy;
                ld_lds2(sH + 2 * pos4(lc, hf, u), hx, hy);
                vx += (TC)wh[u] * (hx - hx0);
                vy += (TC)wh[u] * (hy - hy0);
            }
        }
    }
    if (i < a.N) {
        const TC G = (TC)a.g;
        if (!a.te) {
            const TC A = (TC)a.a;
            S::st2(a.out, i, hx0 + A * (-dy + G * vx), hy0 + A * (dx + G * vy));
        } else {
            // TEz (Ex, Ey) <- E + kappa (D^dy Hz + gamma HV, -D^dx Hz + gamma HV),
            // written as E - kappa (-D^dy Hz - gamma HV, D^dx Hz - gamma HV) with
            // the host's gamma negated; then the wall mask
            const TC A = -kappa_of(a, i);
            TC ex = hx0 + A * (-dy + G * vx), ey = hy0 + A * (dx + G * vy);
            te_wall(a.emask[i], a.wnrm, i, ex, ey);
            S::st2(a.out, i, ex, ey);
        }
    }
}

template <typename TS, typename TW>
__global__ __launch_bounds__(256) void k_e2l(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    using WV = typename WF<TW>::V;
    TC* sE = lds_base<TC>();
    TC* sH = sE + ((a.hmax + 3) & ~3);
    const int wg = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int h0 = a.hoff[wg], hc = a.hoff[wg + 1] - h0;
    stage_rounds<4, Val3<TC>>(
        a.hpool + h0, hc,
        [&](int j) {
            Val3<TC> v;
            v.x = S::ld1(a.E, j);
            S::ld2(a.H, j, v.y, v.z);
            return v;
        },
        [&](int k, const Val3<TC>& v) {
            sE[k] = v.x;
            st_lds2(sH + 2 * k, v.y, v.z);
        });
    __syncthreads();
    const int64_t tile = (int64_t)wg * (RBFFD_WGT / RBFFD_TILE) + (threadIdx.x >> 6);
    if (tile >= a.tiles) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    const TC e0 = S::ld1(a.E, ic);
    TC hx0, hy0;
    S::ld2(a.H, ic, hx0, hy0);
    TC cu = 0, ve = 0;
    const uint4* pl = a.lidx + tile * a.Q8 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 2 * WF<TW>::CH + lane * WF<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * WF<TW>::CH + lane * WF<TW>::LS;
    const int qm = max(a.C4, a.V4);
    uint4 li = ldu4s(pl);
    WV nx[4] = {0, 0, 0, 0}, ny[4] = {0, 0, 0, 0}, nh[4] = {0, 0, 0, 0};
    load2(pc, ph, 0, a.C4, a.V4, nx, ny, nh);
    for (int q = 0; q < qm; ++q) {
        const uint4 lc = li;
        WV wx[4], wy[4], wh[4];
        copy4(wx, nx); copy4(wy, ny); copy4(wh, nh);
        if (q + 1 < qm) {
            if (((q + 1) & 1) == 0) li = ldu4s(pl + ((q + 1) >> 1) * RBFFD_TILE);
            load2(pc, ph, q + 1, a.C4, a.V4, nx, ny, nh);
        }
        const int hf = q & 1;
        if (q < a.C4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                TC hx, hy;
                ld_lds2(sH + 2 * pos4(lc, hf, u), hx, hy);
                cu += (TC)wx[u] * (hy - hy0) - (TC)wy[u] * (hx - hx0);
            }
        }
        if (q < a.V4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) ve += (TC)wh[u] * (sE[pos4(lc, hf, u)] - e0);
        }
    }
    if (i < a.N) {
        const TC k = kappa_of(a, i);
        const TC v = (a.nomask || (a.emask[i] & 1)) ? e0 + k * (cu + (TC)a.g * ve) : (TC)0;
        S::st1(a.out, i, v);
    }
}

template <typename TS, typename TW>
__global__ __launch_bounds__(RBFFD_WGT_3D_F32) void k_h3l(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    TC* sE = lds_base<TC>();                           // 3 values per entry
    TC* sH = sE + 3 * (int64_t)a.hmax;
    const int wg = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int h0 = a.hoff[wg], hc = a.hoff[wg + 1] - h0;
    stage_rounds<4, Val6<TC>>(
        a.hpool + h0, hc,
        [&](int j) {
            Val6<TC> v;
            S::ld3(a.E, j, v.v[0], v.v[1], v.v[2]);
            S::ld3(a.H, j, v.v[3], v.v[4], v.v[5]);
            return v;
        },
        [&](int k, const Val6<TC>& v) {
            const TC e[3] = {v.v[0], v.v[1], v.v[2]}, hh[3] = {v.v[3], v.v[4], v.v[5]};
            st_lds3(sE + 3 * k, e);
            st_lds3(sH + 3 * k, hh);
        });
    __syncthreads();
    const int64_t tile = (int64_t)wg * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= a.tiles) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    TC ex0, ey0, ez0, hx0, hy0, hz0;
    S::ld3(a.E, ic, ex0, ey0, ez0);
    S::ld3(a.H, ic, hx0, hy0, hz0);
    TC xEy = 0, xEz = 0, yEx = 0, yEz = 0, zEx = 0, zEy = 0, vx = 0, vy = 0, vz = 0;
    const uint4* pl = a.lidx + tile * a.Q8 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 3 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const int qm = max(a.C4, a.V4);
    // chunk q + 1 is loaded while chunk q is summed
    uint4 li = ldu4s(pl);
    TW nx[4] = {0, 0, 0, 0}, ny[4] = {0, 0, 0, 0}, nz[4] = {0, 0, 0, 0}, nh[4] = {0, 0, 0, 0};
    load3(pc, ph, 0, a.C4, a.V4, nx, ny, nz, nh);
    for (int q = 0; q < qm; ++q) {
        const uint4 lc = li;
        TW wx[4], wy[4], wz[4], wh[4];
        copy4(wx, nx); copy4(wy, ny); copy4(wz, nz); copy4(wh, nh);
        if (q + 1 < qm) {
            if (((q + 1) & 1) == 0) li = ldu4s(pl + ((q + 1) >> 1) * RBFFD_TILE);
            load3(pc, ph, q + 1, a.C4, a.V4, nx, ny, nz, nh);
        }
        const int hf = q & 1;
        if (q < a.C4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = pos4(lc, hf, u);
                TC v[3];
                ld_lds3(sE + 3 * k, v);
                const TC ex = v[0] - ex0, ey = v[1] - ey0, ez = v[2] - ez0;
                xEy += (TC)wx[u] * ey; xEz += (TC)wx[u] * ez;
                yEx += (TC)wy[u] * ex; yEz += (TC)wy[u] * ez;
                zEx += (TC)wz[u] * ex; zEy += (TC)wz[u] * ey;
            }
        }
        if (q < a.V4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                TC v[3];
                ld_lds3(sH + 3 * pos4(lc, hf, u), v);
                vx += (TC)wh[u] * (v[0] - hx0);
                vy += (TC)wh[u] * (v[1] - hy0);
                vz += (TC)wh[u] * (v[2] - hz0);
            }
        }
    }
    if (i < a.N) {
        const TC A = (TC)a.a, G = (TC)a.g;
        S::st3(a.out, i, hx0 - A * ((yEz - zEy) - G * vx), hy0 - A * ((zEx - xEz) - G * vy),
               hz0 - A * ((xEy - yEx) - G * vz));
    }
}

template <typename TS, typename TW>
__global__ __launch_bounds__(RBFFD_WGT_3D_F32) void k_e3l(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    TC* sE = lds_base<TC>();
    TC* sH = sE + 3 * (int64_t)a.hmax;
    const int wg = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int h0 = a.hoff[wg], hc = a.hoff[wg + 1] - h0;
    stage_rounds<4, Val6<TC>>(
        a.hpool + h0, hc,
        [&](int j) {
            Val6<TC> v;
            S::ld3(a.E, j, v.v[0], v.v[1], v.v[2]);
            S::ld3(a.H, j, v.v[3], v.v[4], v.v[5]);
            return v;
        },
        [&](int k, const Val6<TC>& v) {
            const TC e[3] = {v.v[0], v.v[1], v.v[2]}, hh[3] = {v.v[3], v.v[4], v.v[5]};
            st_lds3(sE + 3 * k, e);
            st_lds3(sH + 3 * k, hh);
        });
    __syncthreads();
    const int64_t tile = (int64_t)wg * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= a.tiles) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = tile * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    TC ex0, ey0, ez0, hx0, hy0, hz0;
    S::ld3(a.E, ic, ex0, ey0, ez0);
    S::ld3(a.H, ic, hx0, hy0, hz0);
    TC xHy = 0, xHz = 0, yHx = 0, yHz = 0, zHx = 0, zHy = 0, vx = 0, vy = 0, vz = 0;
    const uint4* pl = a.lidx + tile * a.Q8 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tile * a.C4 * 3 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const TW* ph = a.wh + tile * a.V4 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const int qm = max(a.C4, a.V4);
    uint4 li = ldu4s(pl);
    TW nx[4] = {0, 0, 0, 0}, ny[4] = {0, 0, 0, 0}, nz[4] = {0, 0, 0, 0}, nh[4] = {0, 0, 0, 0};
    load3(pc, ph, 0, a.C4, a.V4, nx, ny, nz, nh);
    for (int q = 0; q < qm; ++q) {
        const uint4 lc = li;
        TW wx[4], wy[4], wz[4], wh[4];
        copy4(wx, nx); copy4(wy, ny); copy4(wz, nz); copy4(wh, nh);
        if (q + 1 < qm) {
            if (((q + 1) & 1) == 0) li = ldu4s(pl + ((q + 1) >> 1) * RBFFD_TILE);
            load3(pc, ph, q + 1, a.C4, a.V4, nx, ny, nz, nh);
        }
        const int hf = q & 1;
        if (q < a.C4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = pos4(lc, hf, u);
                TC v[3];
                ld_lds3(sH + 3 * k, v);
                const TC hx = v[0] - hx0, hy = v[1] - hy0, hz = v[2] - hz0;
                xHy += (TC)wx[u] * hy; xHz += (TC)wx[u] * hz;
                yHx += (TC)wy[u] * hx; yHz += (TC)wy[u] * hz;
                zHx += (TC)wz[u] * hx; zHy += (TC)wz[u] * hy;
            }
        }
        if (q < a.V4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                TC v[3];
                ld_lds3(sE + 3 * pos4(lc, hf, u), v);
                vx += (TC)wh[u] * (v[0] - ex0);
                vy += (TC)wh[u] * (v[1] - ey0);
                vz += (TC)wh[u] * (v[2] - ez0);
            }
        }
    }
    if (i < a.N) {
        const TC k = kappa_of(a, i), G = (TC)a.g;
        TC nx = ex0 + k * ((yHz - zHy) + G * vx);
        TC ny = ey0 + k * ((zHx - xHz) + G * vy);
        TC nz = ez0 + k * ((xHy - yHx) + G * vz);
        wall3(a.emask[i], a.wnrm, i, nx, ny, nz);
        S::st3(a.out, i, nx, ny, nz);
    }
}

// ---- 3D, two-phase staging ----------------------------------------------------
// When the halo values of both operands do not fit the LDS budget together
// (FP64), the operand of the curl is staged and summed first, then the same
// LDS holds the operand of the hyperviscosity term.  Every accumulator runs
// over the slots in the same order as in the kernels above, so the results
// are the same.  Workgroups keep their idle wavefronts (a partial last
// workgroup) through both barriers.
template <typename TS>
__device__ __forceinline__ void stage_vec3(const TS* F, const int32_t* list, int hc,
                                           typename Store<TS>::C* s) {
    using S = Store<TS>;
    using TC = typename S::C;
    stage_rounds<4, Val3<TC>>(
        list, hc,
        [&](int j) {
            Val3<TC> v;
            S::ld3(F, j, v.x, v.y, v.z);
            return v;
        },
        [&](int k, const Val3<TC>& v) {
            const TC w[3] = {v.x, v.y, v.z};
            st_lds3(s + 3 * k, w);
        });
}

// curl sums over the curl slots: d_x, d_y, d_z of the staged 3-vector field
// (reference values f0) into the six accumulators c[0..5] =
// (x f_y, x f_z, y f_x, y f_z, z f_x, z f_y)
template <typename TC, typename TW>
__device__ __forceinline__ void curl_sums3(const TC* sF, const uint4* pl, const TW* pc, int C4, const TC (&f0)[3],
                                           TC (&c)[6]) {
    uint4 li = ldu4s(pl);
    TW nx[4] = {0, 0, 0, 0}, ny[4] = {0, 0, 0, 0}, nz[4] = {0, 0, 0, 0}, nh[4];
    load3(pc, (const TW*)nullptr, 0, C4, 0, nx, ny, nz, nh);
    for (int q = 0; q < C4; ++q) {
        const uint4 lc = li;
        TW wx[4], wy[4], wz[4];
        copy4(wx, nx); copy4(wy, ny); copy4(wz, nz);
        if (q + 1 < C4) {
            if (((q + 1) & 1) == 0) li = ldu4s(pl + ((q + 1) >> 1) * RBFFD_TILE);
            load3(pc, (const TW*)nullptr, q + 1, C4, 0, nx, ny, nz, nh);
        }
        const int hf = q & 1;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC v[3];
            ld_lds3(sF + 3 * pos4(lc, hf, u), v);
            const TC fx = v[0] - f0[0], fy = v[1] - f0[1], fz = v[2] - f0[2];
            c[0] += (TC)wx[u] * fy; c[1] += (TC)wx[u] * fz;
            c[2] += (TC)wy[u] * fx; c[3] += (TC)wy[u] * fz;
            c[4] += (TC)wz[u] * fx; c[5] += (TC)wz[u] * fy;
        }
    }
}

// hyperviscosity sums over the HV slots of the staged 3-vector field
template <typename TC, typename TW>
__device__ __forceinline__ void hv_sums3(const TC* sF, const uint4* pl, const TW* ph, int V4, const TC (&f0)[3],
                                         TC (&v3)[3]) {
    uint4 li = ldu4s(pl);
    TW nx[4], ny[4], nz[4], nh[4] = {0, 0, 0, 0};
    load3((const TW*)nullptr, ph, 0, 0, V4, nx, ny, nz, nh);
    for (int q = 0; q < V4; ++q) {
        const uint4 lc = li;
        TW wh[4];
        copy4(wh, nh);
        if (q + 1 < V4) {
            if (((q + 1) & 1) == 0) li = ldu4s(pl + ((q + 1) >> 1) * RBFFD_TILE);
            load3((const TW*)nullptr, ph, q + 1, 0, V4, nx, ny, nz, nh);
        }
        const int hf = q & 1;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            TC v[3];
            ld_lds3(sF + 3 * pos4(lc, hf, u), v);
            v3[0] += (TC)wh[u] * (v[0] - f0[0]);
            v3[1] += (TC)wh[u] * (v[1] - f0[1]);
            v3[2] += (TC)wh[u] * (v[2] - f0[2]);
        }
    }
}

template <typename TS, typename TW>
__global__ __launch_bounds__(RBFFD_WGT_3D_F32) void k_h3p(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    TC* sF = lds_base<TC>();
    const int wg = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int h0 = a.hoff[wg], hc = a.hoff[wg + 1] - h0;
    const int64_t tile = (int64_t)wg * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const bool live = tile < a.tiles;
    const int64_t tl = live ? tile : a.tiles - 1;
    const int lane = threadIdx.x & 63;
    const int64_t i = tl * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    TC e0[3], h0v[3];
    S::ld3(a.E, ic, e0[0], e0[1], e0[2]);
    S::ld3(a.H, ic, h0v[0], h0v[1], h0v[2]);
    TC c[6] = {0, 0, 0, 0, 0, 0}, v[3] = {0, 0, 0};
    const uint4* pl = a.lidx + tl * a.Q8 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tl * a.C4 * 3 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const TW* ph = a.wh + tl * a.V4 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    stage_vec3<TS>(a.E, a.hpool + h0, hc, sF);
    __syncthreads();
    if (live) curl_sums3<TC, TW>(sF, pl, pc, a.C4, e0, c);
    __syncthreads();
    stage_vec3<TS>(a.H, a.hpool + h0, hc, sF);
    __syncthreads();
    if (live) hv_sums3<TC, TW>(sF, pl, ph, a.V4, h0v, v);
    if (live && i < a.N) {
        const TC A = (TC)a.a, G = (TC)a.g;
        // c = (xEy, xEz, yEx, yEz, zEx, zEy)
        S::st3(a.out, i, h0v[0] - A * ((c[3] - c[5]) - G * v[0]), h0v[1] - A * ((c[4] - c[1]) - G * v[1]),
               h0v[2] - A * ((c[0] - c[2]) - G * v[2]));
    }
}

template <typename TS, typename TW>
__global__ __launch_bounds__(RBFFD_WGT_3D_F32) void k_e3p(SA<TS, TW> a) {
    using S = Store<TS>;
    using TC = typename S::C;
    TC* sF = lds_base<TC>();
    const int wg = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int h0 = a.hoff[wg], hc = a.hoff[wg + 1] - h0;
    const int64_t tile = (int64_t)wg * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const bool live = tile < a.tiles;
    const int64_t tl = live ? tile : a.tiles - 1;
    const int lane = threadIdx.x & 63;
    const int64_t i = tl * RBFFD_TILE + lane;
    const int64_t ic = i < a.N ? i : a.N - 1;
    TC e0[3], h0v[3];
    S::ld3(a.E, ic, e0[0], e0[1], e0[2]);
    S::ld3(a.H, ic, h0v[0], h0v[1], h0v[2]);
    TC c[6] = {0, 0, 0, 0, 0, 0}, v[3] = {0, 0, 0};
    const uint4* pl = a.lidx + tl * a.Q8 * RBFFD_TILE + lane;
    const TW* pc = a.wc + tl * a.C4 * 3 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    const TW* ph = a.wh + tl * a.V4 * RBFFD_TILE * 4 + lane * WChunk<TW>::LS;
    stage_vec3<TS>(a.H, a.hpool + h0, hc, sF);
    __syncthreads();
    if (live) curl_sums3<TC, TW>(sF, pl, pc, a.C4, h0v, c);
    __syncthreads();
    stage_vec3<TS>(a.E, a.hpool + h0, hc, sF);
    __syncthreads();
    if (live) hv_sums3<TC, TW>(sF, pl, ph, a.V4, e0, v);
    if (live && i < a.N) {
        const TC k = kappa_of(a, i), G = (TC)a.g;
        // c = (xHy, xHz, yHx, yHz, zHx, zHy)
        TC nx = e0[0] + k * ((c[3] - c[5]) + G * v[0]);
        TC ny = e0[1] + k * ((c[4] - c[1]) + G * v[1]);
        TC nz = e0[2] + k * ((c[0] - c[2]) + G * v[2]);
        wall3(a.emask[i], a.wnrm, i, nx, ny, nz);
        S::st3(a.out, i, nx, ny, nz);
    }
}

// ---- per-step auxiliaries (read the device step counter) --------------------
// src: E[node] += amp * wave[n * S + s] after the bracket (PEC nodes stay 0)
template <typename TS>
__global__ void k_source(TS* E, int FE, int comp, const uint8_t* emask, const double* wn, int S, const int32_t* node,
                         const void* amp, const void* wave, const int32_t* ctr, int step_base) {
    using St = Store<TS>;
    using TC = typename St::C;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t n = (int64_t)(*ctr) + step_base;
    for (int s = 0; s < S; ++s) {
        const int64_t i = node[s];
        const int64_t e = i * FE + comp;
        TC v;
        if (sizeof(TC) == 8) v = ((const double*)amp)[s] * ((const double*)wave)[n * S + s];
        else v = ((const float*)amp)[s] * ((const float*)wave)[n * S + s];
        if (emask[i] & 8) {
            // curved 3D wall: E is already projected on the normal n, so adding
            // the projected source v n_comp n keeps (E + v e_comp) projected
            const double* n = wn + 3 * i;
            for (int c = 0; c < 3; ++c)
                St::st1(E, i * FE + c, St::ld1(E, i * FE + c) + v * (TC)n[comp] * (TC)n[c]);
            continue;
        }
        const TC cur = St::ld1(E, e);
        St::st1(E, e, ((emask[i] >> comp) & 1) ? cur + v : (TC)0);
    }
}

template <typename TS>
__global__ void k_receivers(const TS* E, int FE, int comp, int R, const int32_t* node, void* traces, const int32_t* ctr,
                            int T) {
    using St = Store<TS>;
    using TC = typename St::C;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = *ctr;
    if (r >= R || n >= T) return;
    const TC v = St::ld1(E, (int64_t)node[r] * FE + comp);
    if (sizeof(TC) == 8) ((double*)traces)[(int64_t)n * R + r] = (double)v;
    else ((float*)traces)[(int64_t)n * R + r] = (float)v;
}

__global__ void k_ctr_set(int32_t* ctr, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = v;
}
__global__ void k_ctr_inc(int32_t* ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *ctr += 1;
}

// checkpoint: copy (E, H) into slot n / every when n % every == 0 (2-byte units)
__global__ void k_ckpt(const uint16_t* E, int64_t e2, const uint16_t* H, int64_t h2, char* ck, int64_t slot_bytes,
                       int every, const int32_t* ctr) {
    const int n = *ctr;
    if (n % every) return;
    uint16_t* dst = (uint16_t*)(ck + (int64_t)(n / every) * slot_bytes);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < e2 + h2; g += (int64_t)gridDim.x * blockDim.x)
        dst[g] = g < e2 ? E[g] : H[g - e2];
}

// ---- FP64 reductions --------------------------------------------------------

template <typename TS>
__global__ __launch_bounds__(256) void k_energy1(const TS* E, int64_t NE, int FE, int fe, const TS* Ha, const TS* Hb,
                                                 int64_t NH, int FH, int fh, double wE, double wH, double* part,
                                                 const int32_t* ctr, int every) {
    using St = Store<TS>;
    if (ctr && (*ctr % every)) return;
    __shared__ double sh[256];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NE; i += stride)
        for (int c = 0; c < fe; ++c) {
            const double v = (double)St::ld1(E, i * FE + c);
            acc += wE * v * v;
        }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < NH; i += stride)
        for (int c = 0; c < fh; ++c) {
            const double v = 0.5 * ((double)St::ld1(Ha, i * FH + c) + (double)St::ld1(Hb, i * FH + c));
            acc += wH * v * v;
        }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_reduce2(const double* part, int nparts, double* out, const int32_t* ctr,
                                                 int every) {
    if (ctr && (*ctr % every)) return;
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[ctr ? (*ctr / every) : 0] = sh[0];
}

template <typename TS>
__global__ __launch_bounds__(256) void k_compare1(const TS* F, int64_t N, int FS, int nc, const double* ref,
                                                  double* part) {
    using St = Store<TS>;
    __shared__ double sh[3][256];
    double se[4] = {0, 0, 0, 0}, sr[4] = {0, 0, 0, 0}, mx[4] = {0, 0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
        for (int c = 0; c < nc; ++c) {
            const double f = (double)St::ld1(F, i * FS + c), r = ref[i * nc + c];
            const double e = f - r;
            se[c] += e * e;
            sr[c] += r * r;
            mx[c] = fmax(mx[c], fabs(e));
        }
    for (int c = 0; c < nc; ++c) {
        sh[0][threadIdx.x] = se[c];
        sh[1][threadIdx.x] = sr[c];
        sh[2][threadIdx.x] = mx[c];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) {
                sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
                sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
                sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + s]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            part[(blockIdx.x * nc + c) * 3 + 0] = sh[0][0];
            part[(blockIdx.x * nc + c) * 3 + 1] = sh[1][0];
            part[(blockIdx.x * nc + c) * 3 + 2] = sh[2][0];
        }
        __syncthreads();
    }
}

__global__ void k_compare2(const double* part, int nb, int nc, double* out) {
    const int c = threadIdx.x;
    if (c >= nc) return;
    double se = 0, sr = 0, mx = 0;
    for (int b = 0; b < nb; ++b) {
        se += part[(b * nc + c) * 3 + 0];
        sr += part[(b * nc + c) * 3 + 1];
        mx = fmax(mx, part[(b * nc + c) * 3 + 2]);
    }
    out[c * 3 + 0] = se;
    out[c * 3 + 1] = sr;
    out[c * 3 + 2] = mx;
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side: launching one half step of either kind
// ---------------------------------------------------------------------------
namespace {

template <typename TS, typename TW>
void fill_sa(const rbffd_plan* p, const OpBlock& o, SA<TS, TW>& a, bool hupd) {
    a.idx = (const int4*)o.pidx;
    a.idx_h = (const int4*)o.pidx_h;
    a.pref = o.pref;
    a.wc = (const TW*)o.pwc;
    a.wh = (const TW*)o.pwh;
    a.N = o.Nt;
    a.tiles = o.tiles;
    a.C4 = o.C4;
    a.V4 = o.V4;
    a.S4 = o.S4;
    a.xcd = p->var.xcd;
    a.g = p->gamma;
    a.dt = p->dt;
    a.eps0 = p->p.eps0;
    a.a = hupd ? p->dt / p->p.mu0 : p->dt / p->p.eps0;
    a.emask = p->E.emask;
    a.wnrm = p->E.nrm;
    a.lidx = (const uint4*)o.lidx;
    a.hpool = o.hpool;
    a.hoff = o.hoff;
    a.Q8 = o.Q8;
    a.hmax = o.hmax;
}

template <typename TS, typename TW>
void launch_half(const rbffd_plan* p, bool hupd, const void* E, const void* H, void* out, const void* eps_r,
                 hipStream_t st) {
    // compressed (W22) weights exist only for the 2D collocated kernels
    constexpr bool kW22 = std::is_same<TW, w22>::value;
    const OpBlock& o = hupd ? p->opH : p->opE;
    SA<TS, TW> a{};
    fill_sa(p, o, a, hupd);
    a.E = (const TS*)E;
    a.H = (const TS*)H;
    a.out = (TS*)out;
    a.eps_r = hupd ? nullptr : eps_r;
    if (p->p.pol == RBFFD_POL_TE) {
        // TEz: the Hz update runs the scalar (E-update) kernel on (Hz, E) and
        // the E update the vector (H-update) kernel on (Hz_new, E); the
        // scalar kernel's factor is -dt/mu0, both take -gamma
        a.E = (const TS*)H;
        a.H = (const TS*)E;
        a.g = -p->gamma;
        a.a = hupd ? -p->dt / p->p.mu0 : p->dt / p->p.eps0;
        a.nomask = hupd ? 1 : 0;
        a.te = hupd ? 0 : 1;
        hupd = !hupd;
    }
    if (p->collocated && o.hmax > 0 && p->var.lds && !(p->var.lds == 3 && p->dim == 2)) {
        using TC = typename Store<TS>::C;
        const dim3 grid((unsigned)o.nwg), block(o.wgt);
        if (p->dim == 2) {
            const size_t lds = (size_t)(((o.hmax + 3) & ~3) + 2 * o.hmax) * sizeof(TC);
            if (hupd) hipLaunchKernelGGL((k_h2l<TS, TW>), grid, block, lds, st, a);
            else hipLaunchKernelGGL((k_e2l<TS, TW>), grid, block, lds, st, a);
            return;
        }
        if constexpr (kW22) {
            // compressed weights: 2D collocated plans only (refused at plan creation otherwise)
            return;
        } else if (o.stage == 1 && p->var.lds != 2) {
            const size_t lds = (size_t)6 * o.hmax * sizeof(TC);
            if (hupd) hipLaunchKernelGGL((k_h3l<TS, TW>), grid, block, lds, st, a);
            else hipLaunchKernelGGL((k_e3l<TS, TW>), grid, block, lds, st, a);
        } else {
            const size_t lds = (size_t)3 * o.hmax * sizeof(TC);
            if (hupd) hipLaunchKernelGGL((k_h3p<TS, TW>), grid, block, lds, st, a);
            else hipLaunchKernelGGL((k_e3p<TS, TW>), grid, block, lds, st, a);
        }
        return;
    }
    if (p->var.lds == 3 && p->dim == 2 && p->collocated) {
        const dim3 grid((unsigned)o.tiles), block(256);
        if (hupd) hipLaunchKernelGGL((k_h2s<TS, TW>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_e2s<TS, TW>), grid, block, 0, st, a);
        return;
    }
    const int wpb = p->var.block / 64;
    const dim3 grid((unsigned)cdiv(o.tiles, wpb)), block(p->var.block);
    if (p->dim == 2 && p->collocated) {
        if (hupd) hipLaunchKernelGGL((k_h2<TS, TW>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_e2<TS, TW>), grid, block, 0, st, a);
        return;
    }
    if constexpr (!kW22) {
        if (p->dim == 2 && p->var.lds == 3) {
            const dim3 g1((unsigned)o.tiles), b1(256);
            if (hupd) hipLaunchKernelGGL((k_h2xs<TS, TW>), g1, b1, 0, st, a);
            else hipLaunchKernelGGL((k_e2xs<TS, TW>), g1, b1, 0, st, a);
            return;
        }
        if (p->dim == 2) {
            if (hupd) hipLaunchKernelGGL((k_h2x<TS, TW>), grid, block, 0, st, a);
            else hipLaunchKernelGGL((k_e2x<TS, TW>), grid, block, 0, st, a);
        } else {
            if (hupd) hipLaunchKernelGGL((k_h3<TS, TW>), grid, block, 0, st, a);
            else hipLaunchKernelGGL((k_e3<TS, TW>), grid, block, 0, st, a);
        }
    }
}

void half(const rbffd_plan* p, bool hupd, const void* E, const void* H, void* out, const void* eps_r, hipStream_t st) {
    switch (p->p.fdtype) {
        case RBFFD_F64: launch_half<double, double>(p, hupd, E, H, out, eps_r, st); break;
        case RBFFD_F32:
            if (p->p.wdtype == RBFFD_W22) launch_half<float, w22>(p, hupd, E, H, out, eps_r, st);
            else launch_half<float, float>(p, hupd, E, H, out, eps_r, st);
            break;
        default: launch_half<bf16s, float>(p, hupd, E, H, out, eps_r, st); break;
    }
}

template <typename TS>
void launch_energy(const rbffd_plan* p, const void* E, const void* Ha, const void* Hb, double* out, RunWS& w,
                   const int32_t* ctr, int every, hipStream_t st) {
    const double wE = std::pow(p->E.h, p->dim);
    const double hh = p->collocated ? p->E.h : p->H.h;
    const double wH = p->eta0 * p->eta0 * std::pow(hh, p->dim);
    const int64_t nmax = std::max(p->E.N, p->H.N);
    const int nb = (int)std::min<int64_t>(RED_BLOCKS, cdiv(nmax, 256));
    hipLaunchKernelGGL(k_energy1<TS>, dim3(nb), dim3(256), 0, st, (const TS*)E, p->E.N, p->FE, p->fe_comp,
                       (const TS*)Ha, (const TS*)Hb, p->H.N, p->FH, p->fh_comp, wE, wH, w.part, ctr, every);
    hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(256), 0, st, w.part, nb, out, ctr, every);
}

void energy(const rbffd_plan* p, const void* E, const void* Ha, const void* Hb, double* out, RunWS& w,
            const int32_t* ctr, int every, hipStream_t st) {
    switch (p->p.fdtype) {
        case RBFFD_F64: launch_energy<double>(p, E, Ha, Hb, out, w, ctr, every, st); break;
        case RBFFD_F32: launch_energy<float>(p, E, Ha, Hb, out, w, ctr, every, st); break;
        default: launch_energy<bf16s>(p, E, Ha, Hb, out, w, ctr, every, st); break;
    }
}

int check_fields(const rbffd_plan* p, const rbffd_fields* f) {
    if (!f) return set_err(p, RBFFD_EINVAL, "null fields");
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    if (f->cur != 0 && f->cur != 1) return set_err(p, RBFFD_EINVAL, "fields.cur must be 0 or 1");
    for (int b = 0; b < 2; ++b)
        if (!f->E[b] || !f->H[b]) return set_err(p, RBFFD_EINVAL, "null field buffer");
    if (f->E[0] == f->E[1] || f->H[0] == f->H[1]) return set_err(p, RBFFD_EINVAL, "ping-pong buffers must differ");
    return RBFFD_OK;
}

}  // namespace

// K-field batch (batched.hip)
int batched_step(const rbffd_plan* p, rbffd_fields* f, int32_t nsteps, hipStream_t st);

extern "C" int rbffd_step(const rbffd_plan* p, rbffd_fields* f, int32_t nsteps, void* stream) {
    if (!p) return RBFFD_EINVAL;
    int rc = check_fields(p, f);
    if (rc) return rc;
    if (nsteps < 0) return set_err(p, RBFFD_EINVAL, "nsteps < 0");
    hipStream_t st = (hipStream_t)stream;
    if (p->K > 1) return batched_step(p, f, nsteps, st);
    for (int s = 0; s < nsteps; ++s) {
        const int c = f->cur, o = 1 - c;
        half(p, true, f->E[c], f->H[c], f->H[o], nullptr, st);
        half(p, false, f->E[c], f->H[o], f->E[o], f->eps_r, st);
        f->cur = o;
    }
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

extern "C" int rbffd_half(const rbffd_plan* p, const rbffd_fields* f, int32_t which, void* stream) {
    if (!p) return RBFFD_EINVAL;
    int rc = check_fields(p, f);
    if (rc) return rc;
    if (p->K > 1) return set_err(p, RBFFD_ENOTSUP, "rbffd_half is for single-field plans");
    if (which != 0 && which != 1) return set_err(p, RBFFD_EINVAL, "which must be 0 (H) or 1 (E)");
    const int c = f->cur, o = 1 - c;
    if (which == 0) half(p, true, f->E[c], f->H[c], f->H[o], nullptr, (hipStream_t)stream);
    else half(p, false, f->E[c], f->H[o], f->E[o], f->eps_r, (hipStream_t)stream);
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

namespace {
// One full step with every auxiliary; buffers (c -> o) fixed so it can be
// captured.  The device counter holds the step index.
void full_step(const rbffd_plan* p, const rbffd_fields* f, int c, const rbffd_run_args* a, RunWS& w, hipStream_t st) {
    const int o = 1 - c;
    const int comp = p->dim == 2 ? 0 : 2;
    if (a->ckpt) {
        const int64_t eb = p->E.N * p->FE * (int64_t)field_elem_bytes(p->p.fdtype);
        const int64_t hb = p->H.N * p->FH * (int64_t)field_elem_bytes(p->p.fdtype);
        hipLaunchKernelGGL(k_ckpt, dim3(1024), dim3(256), 0, st, (const uint16_t*)f->E[c], eb / 2,
                           (const uint16_t*)f->H[c], hb / 2, (char*)a->ckpt, eb + hb, a->ckpt_every,
                           (const int32_t*)w.ctr);
    }
    half(p, true, f->E[c], f->H[c], f->H[o], nullptr, st);
    if (a->energy_out && a->energy_every > 0)
        energy(p, f->E[c], f->H[c], f->H[o], a->energy_out, w, w.ctr, a->energy_every, st);
    half(p, false, f->E[c], f->H[o], f->E[o], f->eps_r, st);
    if (a->n_src > 0) {
        switch (p->p.fdtype) {
            case RBFFD_F64:
                hipLaunchKernelGGL(k_source<double>, dim3(1), dim3(64), 0, st, (double*)f->E[o], p->FE, comp, p->E.emask,
                                   p->E.nrm, a->n_src, a->src_node, a->src_amp, a->src_wave, w.ctr, a->step0);
                break;
            case RBFFD_F32:
                hipLaunchKernelGGL(k_source<float>, dim3(1), dim3(64), 0, st, (float*)f->E[o], p->FE, comp, p->E.emask,
                                   p->E.nrm, a->n_src, a->src_node, a->src_amp, a->src_wave, w.ctr, a->step0);
                break;
            default:
                hipLaunchKernelGGL(k_source<bf16s>, dim3(1), dim3(64), 0, st, (bf16s*)f->E[o], p->FE, comp,
                                   p->E.emask, p->E.nrm, a->n_src, a->src_node, a->src_amp, a->src_wave, w.ctr, a->step0);
        }
    }
    if (a->n_rcv > 0) {
        const dim3 g((unsigned)cdiv(a->n_rcv, 64));
        switch (p->p.fdtype) {
            case RBFFD_F64:
                hipLaunchKernelGGL(k_receivers<double>, g, dim3(64), 0, st, (const double*)f->E[o], p->FE, comp,
                                   a->n_rcv, a->rcv_node, a->traces, w.ctr, a->T);
                break;
            case RBFFD_F32:
                hipLaunchKernelGGL(k_receivers<float>, g, dim3(64), 0, st, (const float*)f->E[o], p->FE, comp, a->n_rcv,
                                   a->rcv_node, a->traces, w.ctr, a->T);
                break;
            default:
                hipLaunchKernelGGL(k_receivers<bf16s>, g, dim3(64), 0, st, (const bf16s*)f->E[o], p->FE, comp,
                                   a->n_rcv, a->rcv_node, a->traces, w.ctr, a->T);
        }
    }
    // the step counter only feeds the auxiliary kernels
    if (a->ckpt || a->n_src > 0 || a->n_rcv > 0 || (a->energy_out && a->energy_every > 0))
        hipLaunchKernelGGL(k_ctr_inc, dim3(1), dim3(64), 0, st, w.ctr);
}
}  // namespace

int batched_run(const rbffd_plan* p, rbffd_fields* f, const rbffd_run_args* a, void* ws, hipStream_t st);

extern "C" int rbffd_run(const rbffd_plan* p, rbffd_fields* f, const rbffd_run_args* a, void* ws, void* stream) {
    if (!p || !a) return RBFFD_EINVAL;
    int rc = check_fields(p, f);
    if (rc) return rc;
    if (!ws) return set_err(p, RBFFD_EINVAL, "run needs the workspace");
    if (a->T < 0) return set_err(p, RBFFD_EINVAL, "T < 0");
    hipStream_t st = (hipStream_t)stream;
    if (p->K > 1) return batched_run(p, f, a, ws, st);
    if (p->p.pol == RBFFD_POL_TE && (a->n_src > 0 || a->n_rcv > 0))
        return set_err(p, RBFFD_ENOTSUP, "sources and receivers are implemented for TMz");
    if (a->n_src > 0 && (!a->src_node || !a->src_amp || !a->src_wave))
        return set_err(p, RBFFD_EINVAL, "sources need node, amplitude and waveform arrays");
    if (a->n_rcv > 0 && (!a->rcv_node || !a->traces)) return set_err(p, RBFFD_EINVAL, "receivers need nodes and traces");
    if (a->ckpt && a->ckpt_every <= 0) return set_err(p, RBFFD_EINVAL, "ckpt_every must be positive");
    if (a->energy_out && a->energy_every < 0) return set_err(p, RBFFD_EINVAL, "energy_every < 0");
    const int64_t eb = p->E.N * p->FE * (int64_t)field_elem_bytes(p->p.fdtype);
    const int64_t hb = p->H.N * p->FH * (int64_t)field_elem_bytes(p->p.fdtype);
    RunWS w = run_ws(ws);
    hipLaunchKernelGGL(k_ctr_set, dim3(1), dim3(64), 0, st, w.ctr, 0);
    int s = 0;
    if (a->use_graph) {
        rc = replay_steps(
            p, a->T, f->cur, st, [&](int c, hipStream_t cs) { full_step(p, f, c, a, w, cs); }, &s);
        if (rc) return rc;
    }
    int c = f->cur;
    if (s > 0 && (s % 2)) c = 1 - c;
    for (; s < a->T; ++s) {
        full_step(p, f, c, a, w, st);
        c = 1 - c;
    }
    f->cur = (a->T % 2) ? 1 - f->cur : f->cur;
    HIPCHK(p, hipGetLastError());
    if (a->energy_out && a->energy_every > 0 && a->unstable_threshold > 0 && a->T > 0) {
        const int ne = (a->T - 1) / a->energy_every + 1;
        std::vector<double> e(ne);
        HIPCHK(p, hipMemcpyAsync(e.data(), a->energy_out, ne * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(p, hipStreamSynchronize(st));
        for (int k = 0; k < ne; ++k)
            if (!std::isfinite(e[k]) || e[k] > a->unstable_threshold * e[0])
                return set_err(p, RBFFD_EUNSTABLE, "energy sample " + std::to_string(k) + " = " + std::to_string(e[k]) +
                                                       " exceeds the threshold");
    }
    return RBFFD_OK;
}

extern "C" int rbffd_energy(const rbffd_plan* p, const void* E, const void* Ha, const void* Hb, double* out, void* ws,
                            void* stream) {
    if (!p || !E || !Ha || !Hb || !out || !ws) return RBFFD_EINVAL;
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    if (p->K > 1) return set_err(p, RBFFD_ENOTSUP, "energy of a K-field batch: use rbffd_compare per field");
    RunWS w = run_ws(ws);
    energy(p, E, Ha, Hb, out, w, nullptr, 1, (hipStream_t)stream);
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

// ---- energy without a workspace ------------------------------------------------
// rbffd_energy_static runs the same two kernels as rbffd_energy, with the
// per-block FP64 partial sums in this file-scope device array instead of the
// caller's workspace.  Every device holds its own copy at its own address;
// host code uses only that address (looked up once per device), never the
// array's name.  The reduction writes partial b for every block b < nb before
// the second kernel reads partials 0 .. nb - 1, so nothing must start at zero;
// calls that overlap on one device share the array and race.
namespace {
constexpr int kStaticParts = RED_BLOCKS;   // 8 KB of partial sums per device
static __device__ __align__(256) double energy_scratch[kStaticParts];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

int scratch_for(const rbffd_plan* p, hipStream_t st, double** out) {
    int dev = -1;
    if (st) {
        HIPCHK(p, hipStreamGetDevice(st, &dev));
    } else {
        HIPCHK(p, hipGetDevice(&dev));
    }
    if (dev < 0 || dev >= kMaxDevices) return set_err(p, RBFFD_ESIZE, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        HIPCHK(p, hipGetDevice(&cur));
        if (cur != dev) HIPCHK(p, hipSetDevice(dev));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(energy_scratch));
        if (cur != dev) HIPCHK(p, hipSetDevice(cur));
        if (e != hipSuccess || !ptr)
            return set_err(p, RBFFD_EHIP, std::string("hipGetSymbolAddress(energy_scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return RBFFD_OK;
}
}  // namespace

extern "C" int rbffd_energy_static(const rbffd_plan* p, const void* E, const void* Ha, const void* Hb, double* out,
                                   void* stream) {
    if (!p || !E || !Ha || !Hb || !out) return RBFFD_EINVAL;
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    if (p->K > 1) return set_err(p, RBFFD_ENOTSUP, "energy of a K-field batch: use rbffd_compare per field");
    const int64_t nmax = std::max(p->E.N, p->H.N);
    if (std::min<int64_t>(RED_BLOCKS, cdiv(nmax, 256)) > kStaticParts)
        return set_err(p, RBFFD_ESIZE, "more reduction blocks than the static scratch holds");
    hipStream_t st = (hipStream_t)stream;
    double* parts = nullptr;
    int rc = scratch_for(p, st, &parts);
    if (rc) return rc;
    RunWS w{};
    w.part = parts;
    energy(p, E, Ha, Hb, out, w, nullptr, 1, st);
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

extern "C" int rbffd_compare(const rbffd_plan* p, int32_t which, const void* F, const double* ref, double* out,
                             void* ws, void* stream) {
    if (!p || !F || !ref || !out || !ws) return RBFFD_EINVAL;
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    hipStream_t st = (hipStream_t)stream;
    RunWS w = run_ws(ws);
    const bool isE = which == 0;
    const int64_t N = (isE ? p->E.N : p->H.N) * (p->K > 1 ? 1 : 1);
    int FS = isE ? p->FE : p->FH;
    int nc = isE ? p->fe_comp : p->fh_comp;
    int64_t rows = N;
    if (p->K > 1) {
        // batch layout [N][F][K]: compare every (node, comp, k) value as its own row
        rows = N * nc * p->K;
        FS = 1;
        nc = 1;
    }
    const int nb = (int)std::min<int64_t>(RED_BLOCKS, cdiv(rows, 256));
    switch (p->p.fdtype) {
        case RBFFD_F64:
            hipLaunchKernelGGL(k_compare1<double>, dim3(nb), dim3(256), 0, st, (const double*)F, rows, FS, nc, ref, w.part);
            break;
        case RBFFD_F32:
            hipLaunchKernelGGL(k_compare1<float>, dim3(nb), dim3(256), 0, st, (const float*)F, rows, FS, nc, ref, w.part);
            break;
        default:
            hipLaunchKernelGGL(k_compare1<bf16s>, dim3(nb), dim3(256), 0, st, (const bf16s*)F, rows, FS, nc, ref, w.part);
    }
    hipLaunchKernelGGL(k_compare2, dim3(1), dim3(64), 0, st, w.part, nb, nc, out);
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

// ---------------------------------------------------------------------------
// Launch tuning: workgroup size and the XCD remap, timed on the device
// ---------------------------------------------------------------------------
extern "C" int rbffd_autotune(rbffd_plan* p, rbffd_fields* f, int32_t reps, void* stream) {
    if (!p) return RBFFD_EINVAL;
    int rc = check_fields(p, f);
    if (rc) return rc;
    if (reps < 1) reps = 1;
    hipStream_t st = (hipStream_t)stream;
    // candidate launch variants: single field -- workgroup size x XCD remap
    // for the global-gather kernels, plus the LDS-staged kernels (fixed
    // shape) with and without the remap; K-field batch -- workgroup size x
    // resident workgroups per CU for the global kernels, plus the staged one
    std::vector<Variant> cand;
    const bool staged = p->collocated && p->opH.hmax > 0;
    for (int b : {64, 128, 256, 512}) {
        if (p->K > 1) {
            if (b > 256) continue;
            for (int pe : {4, 8, 16}) cand.push_back(Variant{b, 1, pe, 0});
        } else {
            for (int x : {0, 1}) cand.push_back(Variant{b, x, 8, 0});
        }
    }
    if (staged) {
        if (p->K > 1) {
            // staged batch: 4-field (persist < 8), 8-field or 16-field slices,
            // one item per workgroup or persistent with staging wavefronts
            for (int l : {1, 2})
                for (int pe : {4, 8, 16}) cand.push_back(Variant{256, 1, pe, l});
        } else {
            for (int x : {0, 1}) cand.push_back(Variant{256, x, 8, 1});
            // 3D with both operands fitting: also the one-operand-at-a-time kernels
            if (p->dim == 3 && p->opH.stage == 1) cand.push_back(Variant{256, 1, 8, 2});
        }
    }
    if (p->K == 1 && p->dim == 2) {
        // four wavefronts per 64-node tile (small node sets), collocated or two sets
        for (int x : {0, 1}) cand.push_back(Variant{256, x, 8, 3});
    }
    Variant best = p->var;
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    HIPCHK(p, hipEventCreate(&e0));
    HIPCHK(p, hipEventCreate(&e1));
    for (const Variant& v : cand) {
        p->var = v;
        rc = rbffd_step(p, f, 2, stream);   // warm
        if (rc) break;
        HIPCHK(p, hipEventRecord(e0, st));
        rc = rbffd_step(p, f, reps, stream);
        if (rc) break;
        HIPCHK(p, hipEventRecord(e1, st));
        HIPCHK(p, hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(p, hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->var = best;
    return rc;
}
