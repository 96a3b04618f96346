// Discrete adjoint of the 2D TMz leapfrog (collocated), with sqrt(T)-style
// checkpointing and deterministic recomputation.
//
// Forward step n (Kolar-Pozun & Kosec, arXiv 2508.18205, eq. 19, with the
// per-node eps_r, PEC projector P and soft sources of this library):
//   H^{n+1} = (I + B) H^n + A E^n,        A = a [-D^dy; D^dx],  B = a gamma D^hv
//   E^{n+1} = P[(I + K G) E^n + K C H^{n+1} + s^{n+1}],
//   C = [-D^dy, D^dx], G = gamma D^hv, K = diag(dt / (eps0 eps_r)).
// Reverse step n (mu = P lambda_E^{n+1}):
//   lamH_hat   = lambda_H^{n+1} + C^T K mu
//   lambda_E^n = mu + G^T K mu + A^T lamH_hat + r^n     (r^n: receiver residual of E^n)
//   lambda_H^n = (I + B^T) lamH_hat
//   dJ/deps_r,i += -(mu_i / eps_r,i) (E^{n+1}_i - E^n_i - s^{n+1}_i)
//   dJ/da_s     += g_s^n mu_{node_s}
// The transposed operators are gathered from a sliced-ELL copy of D^T built
// at set-up (entries sorted by (row, source, slot)), so the reverse sweep uses
// no atomics and is bitwise reproducible; the checkpointed gradient therefore
// equals the store-everything gradient bit for bit.
#include <algorithm>
#include <vector>

#include "common.h"
#include "fields.h"

namespace {

template <typename T>
struct AA {
    int64_t N, tiles;
    const int64_t* toff;
    const int32_t* twidth;
    const int32_t* tsrc;
    const T* tw;          // [3][tcap]: D^dx, D^dy, D^hv weights of each entry
    int64_t tcap;
    double a, g, dt, eps0;
    const void* eps_r;
    const uint8_t* emask;
    // state
    const T* lamE;        // lambda_E^{n+1}
    const T* lamH;        // lambda_H^{n+1} [N][2]
    T* mu;
    T* kmu;
    T* lhat;              // [N][2]
    T* tmpE;
    T* lamE_out;
    T* lamH_out;          // [N][2]
    const T* En1;         // E^{n+1}
    const T* En;          // E^n
    double* geps;
};

template <typename T>
__device__ __forceinline__ double eps_of(const AA<T>& a, int64_t i) {
    if (!a.eps_r) return 1.0;
    return sizeof(T) == 8 ? ((const double*)a.eps_r)[i] : (double)((const float*)a.eps_r)[i];
}

// mu = P lambda_E, K mu, and the eps_r gradient (source term corrected later)
template <typename T>
__global__ void k_adj1(AA<T> a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const bool free_ = a.emask[i] & 1;
    const T mu = free_ ? a.lamE[i] : (T)0;
    const double er = eps_of(a, i);
    const T kap = (T)(a.dt / (a.eps0 * er));
    a.mu[i] = mu;
    a.kmu[i] = kap * mu;
    if (free_) a.geps[i] += -((double)mu / er) * ((double)a.En1[i] - (double)a.En[i]);
}

// lamH_hat = lambda_H + C^T K mu ; tmpE = mu + gamma D^hv^T K mu
template <typename T>
__global__ void k_adj2(AA<T> a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t t = g >> 6;
    if (t >= a.tiles) return;
    const int l = (int)(g & 63);
    const int64_t j = g;
    const int w = a.twidth[t];
    const int64_t base = a.toff[t] + l;
    T sx = 0, sy = 0, sh = 0;
    for (int q = 0; q < w; ++q) {
        const int64_t e = base + (int64_t)q * 64;
        const int32_t i = a.tsrc[e];
        const T km = a.kmu[i];
        sx += a.tw[e] * km;
        sy += a.tw[a.tcap + e] * km;
        sh += a.tw[2 * a.tcap + e] * km;
    }
    if (j >= a.N) return;
    a.lhat[j * 2 + 0] = a.lamH[j * 2 + 0] - sy;
    a.lhat[j * 2 + 1] = a.lamH[j * 2 + 1] + sx;
    a.tmpE[j] = a.mu[j] + (T)a.g * sh;
}

// lambda_E^n = tmpE + a (-D^dy^T lhx + D^dx^T lhy) ; lambda_H^n = lamH_hat + a gamma D^hv^T lamH_hat
template <typename T>
__global__ void k_adj3(AA<T> a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t t = g >> 6;
    if (t >= a.tiles) return;
    const int l = (int)(g & 63);
    const int64_t j = g;
    const int w = a.twidth[t];
    const int64_t base = a.toff[t] + l;
    T ce = 0, hx = 0, hy = 0;
    for (int q = 0; q < w; ++q) {
        const int64_t e = base + (int64_t)q * 64;
        const int32_t i = a.tsrc[e];
        const T lx = a.lhat[(int64_t)i * 2 + 0], ly = a.lhat[(int64_t)i * 2 + 1];
        const T wx = a.tw[e], wy = a.tw[a.tcap + e], wh = a.tw[2 * a.tcap + e];
        ce += -wy * lx + wx * ly;
        hx += wh * lx;
        hy += wh * ly;
    }
    if (j >= a.N) return;
    const T A = (T)a.a, AG = (T)(a.a * a.g);
    a.lamE_out[j] = a.tmpE[j] + A * ce;
    a.lamH_out[j * 2 + 0] = a.lhat[j * 2 + 0] + AG * hx;
    a.lamH_out[j * 2 + 1] = a.lhat[j * 2 + 1] + AG * hy;
}

// sources: amplitude gradient and the s^{n+1} term of the eps_r gradient;
// receivers: residual injection r^n (n >= 1).  One thread, fixed order.
template <typename T>
__global__ void k_adj_src_rcv(int n, int S, const int32_t* snode, const T* samp, const T* swave, const T* mu,
                              const void* eps_r, double* geps, double* gamp, int R, const int32_t* rnode,
                              const T* gtr, T* lamE, const uint8_t* emask) {
    if (threadIdx.x || blockIdx.x) return;
    for (int s = 0; s < S; ++s) {
        const int64_t i = snode[s];
        const double g = (double)swave[(int64_t)n * S + s];
        gamp[s] += g * (double)mu[i];
        if (emask[i] & 1) {
            const double er = eps_r ? (sizeof(T) == 8 ? ((const double*)eps_r)[i] : (double)((const float*)eps_r)[i]) : 1.0;
            geps[i] += ((double)mu[i] / er) * ((double)samp[s] * g);
        }
    }
    if (n >= 1)
        for (int r = 0; r < R; ++r) lamE[rnode[r]] += gtr[(int64_t)(n - 1) * R + r];
}

template <typename T>
__global__ void k_adj_init(T* lamE, T* lamH, int64_t N, double* geps, double* gamp, int S) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        lamE[i] = 0;
        lamH[2 * i] = 0;
        lamH[2 * i + 1] = 0;
        geps[i] = 0.0;
    }
    if (i < S) gamp[i] = 0.0;
}

template <typename T>
__global__ void k_adj_terminal(T* lamE, int R, const int32_t* rnode, const T* gtr, int T_) {
    if (threadIdx.x || blockIdx.x) return;
    for (int r = 0; r < R; ++r) lamE[rnode[r]] += gtr[(int64_t)(T_ - 1) * R + r];
}

__global__ void k_set_ctr(int32_t* c, int v) {
    if (!threadIdx.x && !blockIdx.x) *c = v;
}

template <typename T>
__global__ void k_src_fwd(T* E, const uint8_t* emask, int S, const int32_t* node, const T* amp, const T* wave, int n) {
    if (threadIdx.x || blockIdx.x) return;
    for (int s = 0; s < S; ++s) {
        const int64_t i = node[s];
        E[i] = (emask[i] & 1) ? E[i] + amp[s] * wave[(int64_t)n * S + s] : (T)0;
    }
}

template <typename T>
int adjoint_impl(const rbffd_plan* p, const rbffd_fields* f, const rbffd_adjoint_args* x, hipStream_t st) {
    const int64_t N = p->E.N;
    const OpBlock& o = p->opH;
    const int64_t eb = N * sizeof(T), hb = 2 * N * sizeof(T);
    char* w = (char*)x->workspace;
    auto take = [&](int64_t bytes) {
        char* r = w;
        w += align_up(bytes, 256);
        return r;
    };
    T* mu = (T*)take(eb);
    T* kmu = (T*)take(eb);
    T* tmpE = (T*)take(eb);
    T* lamE[2] = {(T*)take(eb), (T*)take(eb)};
    T* lamH[2] = {(T*)take(hb), (T*)take(hb)};
    T* lhat = (T*)take(hb);
    T* Ew[2] = {(T*)take(eb), (T*)take(eb)};
    T* Hw[2] = {(T*)take(hb), (T*)take(hb)};
    if (w - (char*)x->workspace > p->adj_ws_bytes) return set_err(p, RBFFD_ESIZE, "adjoint workspace too small");
    T* seg = (T*)x->seg_buf;
    const int C = x->ckpt_every;
    const int T_ = x->T;
    const int nseg = (int)cdiv(T_, C);
    const int B = 256;
    const dim3 gN((unsigned)cdiv(N, B)), gT((unsigned)cdiv(o.tiles * 64, B));

    hipLaunchKernelGGL(k_adj_init<T>, gN, dim3(B), 0, st, lamE[0], lamH[0], N, x->grad_eps, x->grad_amp, x->n_src);
    if (x->n_src > (int64_t)gN.x * B) return set_err(p, RBFFD_ESIZE, "too many sources");
    if (x->n_rcv > 0)
        hipLaunchKernelGGL(k_adj_terminal<T>, dim3(1), dim3(64), 0, st, lamE[0], x->n_rcv, x->rcv_node,
                           (const T*)x->grad_traces, T_);
    int cur = 0;

    rbffd_fields wf{};
    wf.E[0] = Ew[0];
    wf.E[1] = Ew[1];
    wf.H[0] = Hw[0];
    wf.H[1] = Hw[1];
    wf.eps_r = f ? f->eps_r : nullptr;

    AA<T> a{};
    a.N = N;
    a.tiles = o.tiles;
    a.toff = o.t_off;
    a.twidth = o.t_width;
    a.tsrc = o.t_src;
    a.tw = (const T*)o.t_w;
    a.tcap = o.t_cap;
    a.a = p->dt / p->p.mu0;
    a.g = p->gamma;
    a.dt = p->dt;
    a.eps0 = p->p.eps0;
    a.eps_r = wf.eps_r;
    a.emask = p->E.emask;
    a.mu = mu;
    a.kmu = kmu;
    a.lhat = lhat;
    a.tmpE = tmpE;
    a.geps = x->grad_eps;

    for (int k = nseg - 1; k >= 0; --k) {
        const int n0 = k * C, n1 = std::min(T_, n0 + C);
        // restore checkpoint k and recompute E^{n0..n1}
        const char* slot = (const char*)x->ckpt + (int64_t)k * (eb + hb);
        HIPCHK(p, hipMemcpyAsync(Ew[0], slot, eb, hipMemcpyDeviceToDevice, st));
        HIPCHK(p, hipMemcpyAsync(Hw[0], slot + eb, hb, hipMemcpyDeviceToDevice, st));
        HIPCHK(p, hipMemcpyAsync(seg, Ew[0], eb, hipMemcpyDeviceToDevice, st));
        wf.cur = 0;
        for (int n = n0; n < n1; ++n) {
            int rc = rbffd_step(p, &wf, 1, st);
            if (rc) return rc;
            if (x->n_src > 0)
                hipLaunchKernelGGL(k_src_fwd<T>, dim3(1), dim3(64), 0, st, (T*)wf.E[wf.cur], p->E.emask, x->n_src,
                                   x->src_node, (const T*)x->src_amp, (const T*)x->src_wave, n);
            HIPCHK(p, hipMemcpyAsync(seg + (int64_t)(n + 1 - n0) * N, wf.E[wf.cur], eb, hipMemcpyDeviceToDevice, st));
        }
        // reverse sweep over the segment
        for (int n = n1 - 1; n >= n0; --n) {
            a.lamE = lamE[cur];
            a.lamH = lamH[cur];
            a.lamE_out = lamE[1 - cur];
            a.lamH_out = lamH[1 - cur];
            a.En1 = seg + (int64_t)(n + 1 - n0) * N;
            a.En = seg + (int64_t)(n - n0) * N;
            hipLaunchKernelGGL(k_adj1<T>, gN, dim3(B), 0, st, a);
            hipLaunchKernelGGL(k_adj2<T>, gT, dim3(B), 0, st, a);
            hipLaunchKernelGGL(k_adj3<T>, gT, dim3(B), 0, st, a);
            hipLaunchKernelGGL(k_adj_src_rcv<T>, dim3(1), dim3(64), 0, st, n, x->n_src, x->src_node,
                               (const T*)x->src_amp, (const T*)x->src_wave, (const T*)mu, wf.eps_r, x->grad_eps,
                               x->grad_amp, x->n_rcv, x->rcv_node, (const T*)x->grad_traces, lamE[1 - cur], p->E.emask);
            cur = 1 - cur;
        }
    }
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

}  // namespace

extern "C" int rbffd_adjoint(const rbffd_plan* p, const rbffd_fields* f, const rbffd_adjoint_args* x, void* stream) {
    if (!p || !x) return RBFFD_EINVAL;
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    if (!p->p.adjoint) return set_err(p, RBFFD_ENOTSUP, "plan was created without adjoint operators");
    if (x->T < 1 || x->ckpt_every < 1 || !x->ckpt || !x->seg_buf || !x->workspace || !x->grad_eps)
        return set_err(p, RBFFD_EINVAL, "adjoint needs T, ckpt_every, checkpoints, a segment buffer, workspace and grad_eps");
    if (x->n_src > 0 && (!x->src_node || !x->src_amp || !x->src_wave || !x->grad_amp))
        return set_err(p, RBFFD_EINVAL, "sources need node, amplitude, waveform and grad_amp arrays");
    if (x->n_rcv > 0 && (!x->rcv_node || !x->grad_traces)) return set_err(p, RBFFD_EINVAL, "receivers need grad_traces");
    hipStream_t st = (hipStream_t)stream;
    if (p->p.fdtype == RBFFD_F64) return adjoint_impl<double>(p, f, x, st);
    return adjoint_impl<float>(p, f, x, st);
}
