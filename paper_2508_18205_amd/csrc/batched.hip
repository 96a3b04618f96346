// K independent fields sharing one weight set (2D TMz, collocated, FP32).
//
// Fields are stored [N][F][K] (K contiguous).  A wavefront owns one node and
// 64 consecutive fields: the node's stencil indices and weights are
// wave-uniform (scalar loads, read once for all 64 fields) and every
// neighbour gather is one contiguous 256-byte row.  The grid is persistent:
// a fixed number of resident workgroups strides over (node, field-chunk)
// items, so the same wavefront keeps streaming through neighbouring nodes.
// The update is the same eq. 19 step as the single-field kernels
// (Kolar-Pozun & Kosec, arXiv 2508.18205, Section 5), in difference form.
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
    int64_t N;
    int K, KC;            // fields, 64-field chunks
    int S, C, V;          // padded slot counts (multiples of 4)
    float a, g;
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
        float dx = 0.f, dy = 0.f, vx = 0.f, vy = 0.f;
        const int32_t* pi = a.idx + i * a.S;
        const float* px = a.wc + (i * 2 + 0) * a.C;
        const float* py = a.wc + (i * 2 + 1) * a.C;
        const float* ph = a.wh + i * a.V;
        const int both = min(a.C, a.V);
        int s = 0;
        for (; s < both; ++s) {
            const int64_t j = pi[s];
            const float de = a.E[j * K + kk] - e0;
            dx += px[s] * de;
            dy += py[s] * de;
            vx += ph[s] * (a.H[(j * 2 + 0) * K + kk] - hx0);
            vy += ph[s] * (a.H[(j * 2 + 1) * K + kk] - hy0);
        }
        for (; s < a.C; ++s) {
            const int64_t j = pi[s];
            const float de = a.E[j * K + kk] - e0;
            dx += px[s] * de;
            dy += py[s] * de;
        }
        for (; s < a.V; ++s) {
            const int64_t j = pi[s];
            vx += ph[s] * (a.H[(j * 2 + 0) * K + kk] - hx0);
            vy += ph[s] * (a.H[(j * 2 + 1) * K + kk] - hy0);
        }
        if (on) {
            a.out[(i * 2 + 0) * K + k] = hx0 + a.a * (-dy + a.g * vx);
            a.out[(i * 2 + 1) * K + k] = hy0 + a.a * (dx + a.g * vy);
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
        float cu = 0.f, ve = 0.f;
        const int32_t* pi = a.idx + i * a.S;
        const float* px = a.wc + (i * 2 + 0) * a.C;
        const float* py = a.wc + (i * 2 + 1) * a.C;
        const float* ph = a.wh + i * a.V;
        const int both = min(a.C, a.V);
        int s = 0;
        for (; s < both; ++s) {
            const int64_t j = pi[s];
            cu += px[s] * (a.H[(j * 2 + 1) * K + kk] - hy0) - py[s] * (a.H[(j * 2 + 0) * K + kk] - hx0);
            ve += ph[s] * (a.E[j * K + kk] - e0);
        }
        for (; s < a.C; ++s) {
            const int64_t j = pi[s];
            cu += px[s] * (a.H[(j * 2 + 1) * K + kk] - hy0) - py[s] * (a.H[(j * 2 + 0) * K + kk] - hx0);
        }
        for (; s < a.V; ++s) {
            const int64_t j = pi[s];
            ve += ph[s] * (a.E[j * K + kk] - e0);
        }
        if (on) a.out[i * K + k] = (a.emask[i] & 1) ? e0 + a.a * (cu + a.g * ve) : 0.f;
    }
}

BA make_args(const rbffd_plan* p) {
    const OpBlock& o = p->opH;
    BA a{};
    a.idx = o.bidx;
    a.wc = o.bwc;
    a.wh = o.bwh;
    a.N = o.Nt;
    a.K = p->K;
    a.KC = (int)cdiv(p->K, 64);
    a.S = o.S4 * 4;
    a.C = o.C4 * 4;
    a.V = o.V4 * 4;
    a.g = (float)p->gamma;
    a.emask = p->E.emask;
    return a;
}

void launch_pair(const rbffd_plan* p, const rbffd_fields* f, int c, hipStream_t st) {
    const int o = 1 - c;
    BA a = make_args(p);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int wpb = p->var.block / 64;
    const int64_t need = cdiv(a.N * a.KC, wpb);
    const int grid = (int)std::min<int64_t>(need, (int64_t)cus * p->var.persist);
    a.E = (const float*)f->E[c];
    a.H = (const float*)f->H[c];
    a.out = (float*)f->H[o];
    a.a = (float)(p->dt / p->p.mu0);
    hipLaunchKernelGGL(k_hb, dim3(grid), dim3(p->var.block), 0, st, a);
    a.H = (const float*)f->H[o];
    a.out = (float*)f->E[o];
    a.a = (float)(p->dt / p->p.eps0);
    hipLaunchKernelGGL(k_eb, dim3(grid), dim3(p->var.block), 0, st, a);
}

}  // namespace

int batched_step(const rbffd_plan* p, rbffd_fields* f, int32_t nsteps, hipStream_t st) {
    if (f->eps_r) return set_err(p, RBFFD_ENOTSUP, "per-node eps_r is not supported for K-field batches");
    if (p->var.block > 256) return set_err(p, RBFFD_EINVAL, "K-field batches use at most 256 threads per workgroup");
    for (int s = 0; s < nsteps; ++s) {
        launch_pair(p, f, f->cur, st);
        f->cur = 1 - f->cur;
    }
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

int batched_run(const rbffd_plan* p, rbffd_fields* f, const rbffd_run_args* a, void*, hipStream_t st) {
    if (a->n_src || a->n_rcv || a->ckpt || (a->energy_out && a->energy_every))
        return set_err(p, RBFFD_ENOTSUP, "K-field batches run without sources, receivers, energy or checkpoints");
    if (f->eps_r) return set_err(p, RBFFD_ENOTSUP, "per-node eps_r is not supported for K-field batches");
    if (p->var.block > 256) return set_err(p, RBFFD_EINVAL, "K-field batches use at most 256 threads per workgroup");
    int s = 0;
    if (a->use_graph && a->T >= 4) {
        hipGraph_t g;
        hipGraphExec_t ge;
        hipStream_t cs;
        int rc = capture_stream(p, &cs);
        if (rc) return rc;
        HIPCHK(p, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        launch_pair(p, f, f->cur, cs);
        launch_pair(p, f, 1 - f->cur, cs);
        HIPCHK(p, hipStreamEndCapture(cs, &g));
        HIPCHK(p, hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        for (; s + 2 <= a->T; s += 2) HIPCHK(p, hipGraphLaunch(ge, st));
        HIPCHK(p, hipGraphExecDestroy(ge));
        HIPCHK(p, hipGraphDestroy(g));
    }
    for (; s < a->T; ++s) {
        launch_pair(p, f, f->cur, st);
        f->cur = 1 - f->cur;
    }
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}
