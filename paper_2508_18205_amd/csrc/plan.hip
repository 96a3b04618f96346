// Plan creation, parameter validation, arena layout and the parity I/O calls.
#include <cmath>
#include <cstring>
#include <algorithm>

#include "common.h"
#include "wpack.h"

int set_err(const rbffd_plan* p, int code, const std::string& msg) {
    if (p) const_cast<rbffd_plan*>(p)->err = msg;
    return code;
}

int64_t n_monomials(int d, int m) {
    // C(m + d, d)
    int64_t r = 1;
    for (int i = 1; i <= d; ++i) r = r * (m + i) / i;
    return r;
}

// Monomials of total degree <= m in graded lexicographic order
// (1, x, y, x^2, xy, y^2, ...; z last in 3D).
void fill_exponents(int d, int m, int ex[RBFFD_MAX_MONO][3]) {
    int q = 0;
    for (int g = 0; g <= m; ++g) {
        if (d == 2) {
            for (int a = g; a >= 0; --a) { ex[q][0] = a; ex[q][1] = g - a; ex[q][2] = 0; ++q; }
        } else {
            for (int a = g; a >= 0; --a)
                for (int b = g - a; b >= 0; --b) { ex[q][0] = a; ex[q][1] = b; ex[q][2] = g - a - b; ++q; }
        }
    }
}

int field_elem_bytes(int t) { return t == RBFFD_F64 ? 8 : (t == RBFFD_F32 ? 4 : 2); }
int weight_elem_bytes(int t) { return t == RBFFD_F64 ? 8 : 4; }

extern "C" const char* rbffd_strerror(int code) {
    switch (code) {
        case RBFFD_OK: return "ok";
        case RBFFD_EINVAL: return "invalid argument";
        case RBFFD_ESIZE: return "size exceeds a supported maximum";
        case RBFFD_ESINGULAR: return "singular local weight system";
        case RBFFD_EHIP: return "HIP runtime error";
        case RBFFD_EUNSTABLE: return "unstable run (NaN/Inf or energy growth)";
        case RBFFD_ESTATE: return "call out of order";
        case RBFFD_ENOTSUP: return "not supported for this plan";
        default: return "unknown error";
    }
}

extern "C" const char* rbffd_last_error(const rbffd_plan* p) { return p ? p->err.c_str() : ""; }

// ---------------------------------------------------------------------------
// Arena layout
// ---------------------------------------------------------------------------
namespace {
struct Bump {
    char* base;
    int64_t off = 0;
    template <typename T>
    T* take(int64_t count, int64_t align = 256) {
        off = align_up(off, align);
        T* r = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * (int64_t)sizeof(T);
        return r;
    }
    void* take_bytes(int64_t bytes, int64_t align = 256) {
        off = align_up(off, align);
        void* r = base ? base + off : nullptr;
        off += bytes;
        return r;
    }
};

void layout_set(Bump& b, NodeSet& S, int dim, bool is_e, bool normals) {
    S.xyz_in = b.take<double>(S.N * dim);
    S.flags_in = b.take<uint8_t>(S.N);
    S.perm = b.take<int32_t>(S.N);
    S.inv = b.take<int32_t>(S.N);
    S.xyz = b.take<double>(S.N * dim);
    S.emask = is_e ? b.take<uint8_t>(S.N) : nullptr;
    S.nrm = normals ? b.take<double>(S.N * dim) : nullptr;
}

void layout_block(Bump& b, OpBlock& o, int dim, int wb, int cb, int K, bool adjoint) {
    o.tiles = cdiv(o.Nt, RBFFD_TILE);
    o.C4 = (int)cdiv(o.n - 1, 4);
    o.V4 = o.nh > 0 ? (int)cdiv(o.nh - 1, 4) : 0;
    o.S4 = std::max(o.C4, o.V4);
    const int64_t T = o.tiles * RBFFD_TILE;
    if (!o.cross) {
        o.st_union = b.take<int32_t>(o.Nt * o.ns);
        o.pidx = b.take_bytes(T * o.S4 * 16);
        // halo lists per workgroup tile: 256 nodes in 2D, in 3D 1024 with
        // FP32 weights (16-byte chunks) and 512 with FP64, 128 in K-field
        // batch plans
        o.Q8 = (int)cdiv(o.ns - 1, 8);
        o.wgt = K > 1 ? RBFFD_WGT_BATCH : (dim == 3 ? (cb == 16 ? RBFFD_WGT_3D_F32 : RBFFD_WGT_3D) : RBFFD_WGT);
        o.nwg = cdiv(o.tiles, o.wgt / RBFFD_TILE);
        o.lidx = b.take<uint16_t>(T * o.Q8 * 8);
        if (K > 1) o.lself = b.take<uint16_t>(T);
        o.hpool = b.take<int32_t>(o.Nt * o.ns);
        o.hoff = b.take<int32_t>(o.nwg + 1);
    } else {
        o.st_curl = b.take<int32_t>(o.Nt * o.n);
        o.st_hv = o.nh > 0 ? b.take<int32_t>(o.Nt * o.nh) : nullptr;
        o.pidx = b.take_bytes(T * o.C4 * 16);
        o.pidx_h = b.take_bytes(T * o.V4 * 16);
        o.pref = b.take<int32_t>(o.Nt);
    }
    o.wc = b.take<double>(o.Nt * dim * o.n);
    o.wh = o.nh > 0 ? b.take<double>(o.Nt * o.nh) : nullptr;
    o.pwc = b.take_bytes(T * o.C4 * dim * cb);
    o.pwh = b.take_bytes(T * std::max(o.V4, 0) * cb);
    if (K > 1) {
        o.bidx = b.take<int32_t>(o.Nt * o.S4 * 4);
        o.bwc = b.take<float>(o.Nt * dim * o.C4 * 4);
        o.bwh = b.take<float>(o.Nt * o.V4 * 4);
        o.bw0 = b.take<float>(o.Nt * 4);
    }
    if (adjoint) {
        o.t_off = b.take<int64_t>(o.tiles + 1);
        o.t_width = b.take<int32_t>(o.tiles);
        // kNN in-degree is bounded by the kissing number times the stencil
        // size (6 in 2D); the SELL rows are padded to their tile's maximum.
        o.t_cap = T * 6 * (int64_t)o.ns;
        o.t_src = b.take<int32_t>(o.t_cap);
        o.t_slot = b.take<int32_t>(o.t_cap);
        o.t_w = b.take_bytes(o.t_cap * 3 * wb);   // [3][t_cap]: D^dx, D^dy, D^hv weights
    }
}
}  // namespace

int64_t layout_arena(rbffd_plan* p, char* base, int64_t* ws, int64_t* adj_ws) {
    Bump b{base};
    const int wb = weight_elem_bytes(p->p.wdtype);
    layout_set(b, p->E, p->dim, true, has_wall_normals(p));
    if (!p->collocated) layout_set(b, p->H, p->dim, false, false);
    const int cb = chunk_bytes(p->p.wdtype);
    layout_block(b, p->opH, p->dim, wb, cb, p->K, p->p.adjoint != 0);
    if (!p->collocated) layout_block(b, p->opE, p->dim, wb, cb, p->K, false);
    else {
        // the E update uses the same operator block
        OpBlock keep = p->opE;
        p->opE = p->opH;
        (void)keep;
    }
    p->gk = p->K > 1 ? b.take<float>(p->K) : nullptr;
    if (ws) *ws = setup_ws_bytes(p);
    if (adj_ws) {
        const int64_t fb = field_elem_bytes(p->p.fdtype) > 4 ? 8 : 4;
        // mu, kappa*mu, tmpE, lambda_E x2, lambda_H x2 (2 comps), lamH_hat (2),
        // recompute state E x2, H x2 (2 comps), plus partial sums
        *adj_ws = align_up(p->E.N * fb * (3 + 2 + 4 + 2 + 2 + 4), 256) + (1 << 16);
    }
    return align_up(b.off, 256);
}

// ---------------------------------------------------------------------------
// Plan creation
// ---------------------------------------------------------------------------
extern "C" int rbffd_plan_create(const rbffd_params* prm, int64_t N, const double* xyz_host,
                                 const uint8_t* flags_host, int64_t N_h, const double* xyzH_host,
                                 const uint8_t* flagsH_host, rbffd_plan** out) {
    if (!prm || !out || !xyz_host) return RBFFD_EINVAL;
    *out = nullptr;
    rbffd_plan* p = new rbffd_plan();
    p->p = *prm;
    const rbffd_params& q = p->p;
    auto fail = [&](int code, const std::string& m) {
        // no plan for the caller to inspect: print the reason once
        fprintf(stderr, "rbffd_plan_create: %s\n", m.c_str());
        delete p;
        return code;
    };
    if (q.dim != 2 && q.dim != 3) return fail(RBFFD_EINVAL, "dim must be 2 or 3");
    if (q.mode < 0 || q.mode > 2) return fail(RBFFD_EINVAL, "unknown mode");
    if (q.mode == RBFFD_MODE_STAG2 && q.dim != 2)
        return fail(RBFFD_ENOTSUP, "the two-set variant is implemented for 2D TMz");
    if (q.phs_k < 3 || (q.phs_k % 2) == 0) return fail(RBFFD_EINVAL, "phs_k must be odd and >= 3");
    if (q.m < 1) return fail(RBFFD_EINVAL, "m must be >= 1 (PHS r^3 is conditionally positive definite of order 2)");
    if (q.hv_alpha < 0 || q.hv_alpha > 3) return fail(RBFFD_ENOTSUP, "hv_alpha must be 0..3");
    if (q.h <= 0) return fail(RBFFD_EINVAL, "h must be positive");
    if (q.eps0 <= 0 || q.mu0 <= 0) return fail(RBFFD_EINVAL, "eps0 and mu0 must be positive");
    if (q.wdtype != RBFFD_F64 && q.wdtype != RBFFD_F32 && q.wdtype != RBFFD_W22)
        return fail(RBFFD_EINVAL, "wdtype must be F64, F32 or W22");
    if (q.wdtype == RBFFD_W22 &&
        (q.fdtype != RBFFD_F32 || q.dim != 2 || q.mode == RBFFD_MODE_STAG2 || q.K != 1 || q.adjoint))
        return fail(RBFFD_ENOTSUP, "W22 weights are implemented for 2D collocated single-field FP32 plans "
                                   "without the adjoint");
    if (q.fdtype < 0 || q.fdtype > 2) return fail(RBFFD_EINVAL, "bad fdtype");
    if (q.fdtype == RBFFD_BF16 && q.wdtype != RBFFD_F32) return fail(RBFFD_EINVAL, "BF16 fields need F32 weights");
    if (q.fdtype == RBFFD_F32 && q.wdtype == RBFFD_F64) return fail(RBFFD_EINVAL, "F32 fields need F32 or W22 weights");
    if (q.fdtype == RBFFD_F64 && q.wdtype != RBFFD_F64) return fail(RBFFD_EINVAL, "F64 fields need F64 weights");
    if (q.bc != RBFFD_BC_PEC && q.bc != RBFFD_BC_PERIODIC) return fail(RBFFD_EINVAL, "bad bc");
    if (q.reorder < 0 || q.reorder > 2) return fail(RBFFD_EINVAL, "bad reorder");
    if (q.K < 1 || q.K > 4096) return fail(RBFFD_EINVAL, "K must be 1..4096");
    if (q.K > 1 && (q.dim != 2 || q.mode == RBFFD_MODE_STAG2 || q.fdtype != RBFFD_F32))
        return fail(RBFFD_ENOTSUP, "K-field batches are implemented for collocated 2D FP32");
    if (q.adjoint && (q.dim != 2 || q.mode == RBFFD_MODE_STAG2 || q.K != 1 || q.fdtype == RBFFD_BF16))
        return fail(RBFFD_ENOTSUP, "the adjoint is implemented for collocated 2D, K = 1, F32/F64");
    if (q.pol != RBFFD_POL_TM && q.pol != RBFFD_POL_TE) return fail(RBFFD_EINVAL, "pol must be TM or TE");
    if (q.pol == RBFFD_POL_TE && (q.dim != 2 || q.mode == RBFFD_MODE_STAG2 || q.K != 1 || q.adjoint))
        return fail(RBFFD_ENOTSUP, "the TEz polarisation is implemented for collocated 2D, K = 1, no adjoint");
    if (!std::isfinite(q.frame_angle) || (q.dim != 2 && q.frame_angle != 0.0))
        return fail(RBFFD_EINVAL, "frame_angle must be finite, and 0 unless dim = 2");
    if (q.frame_angle != 0.0 && q.pol == RBFFD_POL_TE && q.bc == RBFFD_BC_PEC)
        return fail(RBFFD_ENOTSUP, "TEz walls are axis-aligned: a rotated frame needs periodic boundaries");
    if (N < 1 || N > (int64_t)INT32_MAX / 2) return fail(RBFFD_ESIZE, "N out of range");
    for (int k = 0; k < q.dim; ++k)
        if (!(q.hi[k] > q.lo[k])) return fail(RBFFD_EINVAL, "hi must exceed lo on every axis");

    p->dim = q.dim;
    p->collocated = q.mode != RBFFD_MODE_STAG2;
    p->K = q.K;
    // K-field batches start on the staged kernels with 16-field slices where
    // K and the LDS allow (the tuner's usual choice), else 8 or 4
    if (q.K > 1) p->var.persist = 16;
    p->n = q.n;
    p->M = (int)n_monomials(q.dim, q.m);
    if (p->M > RBFFD_MAX_MONO) return fail(RBFFD_ESIZE, "too many monomials for the curl system");
    if (q.n <= p->M) return fail(RBFFD_EINVAL, "n must exceed the number of monomials M_m");
    if (q.hv_alpha > 0) {
        p->Mh = (int)n_monomials(q.dim, 2 * q.hv_alpha);
        if (p->Mh > RBFFD_MAX_MONO) return fail(RBFFD_ESIZE, "too many monomials for the HV system");
        p->nh = q.n_hv > 0 ? q.n_hv : 2 * p->Mh + 1;
        if (p->nh <= p->Mh) return fail(RBFFD_EINVAL, "n_hv must exceed M_{2 alpha}");
    } else {
        p->nh = 0;
    }
    p->ns = std::max(p->n, p->nh);
    if (p->ns > RBFFD_MAX_STENCIL) return fail(RBFFD_ESIZE, "stencil larger than 128");
    fill_exponents(q.dim, q.m, p->ex_m);
    if (q.hv_alpha > 0) fill_exponents(q.dim, 2 * q.hv_alpha, p->ex_h);

    p->c0 = 1.0 / std::sqrt(q.eps0 * q.mu0);
    p->eta0 = std::sqrt(q.mu0 / q.eps0);
    p->dt = q.dt > 0 ? q.dt : q.h / (10.0 * std::sqrt(2.0) * p->c0);
    if (q.hv_alpha > 0) {
        const double sgn = (q.hv_alpha - 1) % 2 == 0 ? 1.0 : -1.0;
        p->hv_fac = sgn * std::pow(q.h, 2 * q.hv_alpha);
        p->gamma = q.hv_c * p->hv_fac;
    }
    if (q.fdtype == RBFFD_F64 || q.fdtype == RBFFD_F32 || q.fdtype == RBFFD_BF16) {
        const bool te = q.pol == RBFFD_POL_TE;
        p->fe_comp = q.dim == 2 ? (te ? 2 : 1) : 3;
        p->fh_comp = q.dim == 2 ? (te ? 1 : 2) : 3;
        p->FE = q.dim == 2 ? (te ? 2 : 1) : 4;
        p->FH = q.dim == 2 ? (te ? 1 : 2) : 4;
    }
    // Morton quantisation box: square, side = largest extent
    double side = 0;
    for (int k = 0; k < q.dim; ++k) { p->mlo[k] = q.lo[k]; side = std::max(side, q.hi[k] - q.lo[k]); }
    p->mside = side;

    p->E.N = N;
    p->E.h = q.h;
    p->E.xyz_host.assign(xyz_host, xyz_host + N * q.dim);
    p->E.flags_host.assign(N, 0);
    if (flags_host && q.bc == RBFFD_BC_PEC) std::memcpy(p->E.flags_host.data(), flags_host, N);
    if (q.bc == RBFFD_BC_PERIODIC) {
        for (int64_t i = 0; i < N; ++i)
            for (int k = 0; k < q.dim; ++k) {
                const double x = xyz_host[i * q.dim + k];
                if (!(x >= q.lo[k] && x < q.hi[k])) return fail(RBFFD_EINVAL, "periodic node outside [lo, hi)");
            }
    }
    if (!p->collocated) {
        if (N_h < 1 || !xyzH_host) return fail(RBFFD_EINVAL, "two-set variant needs the H node set");
        p->H.N = N_h;
        p->H.h = q.h_h > 0 ? q.h_h : q.h;
        p->H.xyz_host.assign(xyzH_host, xyzH_host + N_h * q.dim);
        p->H.flags_host.assign(N_h, 0);
        if (flagsH_host && q.bc == RBFFD_BC_PEC) std::memcpy(p->H.flags_host.data(), flagsH_host, N_h);
        if (q.bc == RBFFD_BC_PERIODIC) {
            for (int64_t i = 0; i < N_h; ++i)
                for (int k = 0; k < q.dim; ++k) {
                    const double x = xyzH_host[i * q.dim + k];
                    if (!(x >= q.lo[k] && x < q.hi[k])) return fail(RBFFD_EINVAL, "periodic H node outside [lo, hi)");
                }
        }
        if (p->n > N_h || p->n > N || p->nh > N || p->nh > N_h) return fail(RBFFD_EINVAL, "stencil larger than a node set");
    } else {
        p->H.N = N;
        if (p->ns > N) return fail(RBFFD_EINVAL, "stencil larger than the node set");
    }
    // operator blocks
    if (p->collocated) {
        p->opH.Nt = N; p->opH.Ns = N; p->opH.n = p->n; p->opH.nh = p->nh; p->opH.ns = p->ns;
        p->opH.cross = false;
    } else {
        p->opH.Nt = p->H.N; p->opH.Ns = N; p->opH.n = p->n; p->opH.nh = p->nh; p->opH.ns = 0; p->opH.cross = true;
        p->opE.Nt = N; p->opE.Ns = p->H.N; p->opE.n = p->n; p->opE.nh = p->nh; p->opE.ns = 0; p->opE.cross = true;
    }
    int64_t ws = 0, aws = 0;
    p->arena_bytes = layout_arena(p, nullptr, &ws, &aws);
    // run workspace: reduction partials and counters
    p->ws_bytes = std::max<int64_t>(ws, 1 << 20);
    p->adj_ws_bytes = aws;
    *out = p;
    return RBFFD_OK;
}

extern "C" int rbffd_set_wall_normals(rbffd_plan* p, const double* normals_host) {
    if (!p) return RBFFD_EINVAL;
    if (p->p.bc != RBFFD_BC_PEC || !(p->p.pol == RBFFD_POL_TE || p->dim == 3) || !p->collocated)
        return set_err(p, RBFFD_ENOTSUP, "wall normals apply to collocated TEz or 3D plans with PEC walls");
    if (p->ready) return set_err(p, RBFFD_ESTATE, "wall normals must be set before rbffd_weights");
    const int64_t N = p->E.N;
    const int d = p->dim;
    if (!normals_host) {
        p->E.nrm_host.clear();
        return RBFFD_OK;
    }
    for (int64_t i = 0; i < N; ++i) {
        double n2 = 0.0;
        bool finite = true, zero = true;
        for (int k = 0; k < d; ++k) {
            const double v = normals_host[d * i + k];
            finite = finite && std::isfinite(v);
            zero = zero && v == 0.0;
            n2 += v * v;
        }
        if (zero) continue;
        if (!finite || std::fabs(n2 - 1.0) > 1e-9)
            return set_err(p, RBFFD_EINVAL, "wall normal of node " + std::to_string(i) + " is not a unit vector");
        if (p->E.flags_host[i] == 0)
            return set_err(p, RBFFD_EINVAL, "node " + std::to_string(i) + " has a wall normal but no wall flag");
    }
    p->E.nrm_host.assign(normals_host, normals_host + d * N);
    return RBFFD_OK;
}

extern "C" int rbffd_plan_sizes(const rbffd_plan* p, rbffd_sizes* s) {
    if (!p || !s) return RBFFD_EINVAL;
    std::memset(s, 0, sizeof(*s));
    s->N = p->E.N;
    s->N_h = p->H.N;
    s->n_stencil = p->ns;
    s->n_hv = p->nh;
    s->fe = p->FE;
    s->fh = p->FH;
    s->field_elem = field_elem_bytes(p->p.fdtype);
    s->K = p->K;
    s->arena_bytes = p->arena_bytes;
    s->workspace_bytes = p->ws_bytes;
    s->e_bytes = p->E.N * p->FE * p->K * (int64_t)s->field_elem;
    s->h_bytes = p->H.N * p->FH * p->K * (int64_t)s->field_elem;
    s->adjoint_ws_bytes = p->adj_ws_bytes;
    s->dt = p->dt;
    s->gamma = p->gamma;
    return RBFFD_OK;
}

extern "C" void rbffd_plan_destroy(rbffd_plan* p) {
    if (p && p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    delete p;
}

int capture_stream(const rbffd_plan* p, hipStream_t* out) {
    if (!p->cap_stream) HIPCHK(p, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    *out = p->cap_stream;
    return RBFFD_OK;
}

// ---------------------------------------------------------------------------
// Parity I/O
// ---------------------------------------------------------------------------
extern "C" int rbffd_get_perm(const rbffd_plan* p, int32_t set, int32_t* out, void* stream) {
    if (!p || !out) return RBFFD_EINVAL;
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    const NodeSet& S = (set == 1 && !p->collocated) ? p->H : p->E;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(p, hipMemcpyAsync(out, S.perm, S.N * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(p, hipStreamSynchronize(s));
    return RBFFD_OK;
}

extern "C" int rbffd_get_stencils(const rbffd_plan* p, int32_t which, int32_t* out, void* stream) {
    if (!p || !out) return RBFFD_EINVAL;
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    hipStream_t s = (hipStream_t)stream;
    const int32_t* src = nullptr;
    int64_t count = 0;
    if (p->collocated) {
        if (which != RBFFD_ST_UNION) return set_err(p, RBFFD_EINVAL, "collocated plans have one union stencil");
        src = p->opH.st_union;
        count = p->opH.Nt * p->ns;
    } else {
        switch (which) {
            case RBFFD_ST_CURL_H: src = p->opH.st_curl; count = p->opH.Nt * p->n; break;
            case RBFFD_ST_HV_H: src = p->opH.st_hv; count = p->opH.Nt * p->nh; break;
            case RBFFD_ST_CURL_E: src = p->opE.st_curl; count = p->opE.Nt * p->n; break;
            case RBFFD_ST_HV_E: src = p->opE.st_hv; count = p->opE.Nt * p->nh; break;
            default: return set_err(p, RBFFD_EINVAL, "unknown stencil selector");
        }
    }
    if (!src || count == 0) return set_err(p, RBFFD_EINVAL, "stencil not present in this plan");
    HIPCHK(p, hipMemcpyAsync(out, src, count * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(p, hipStreamSynchronize(s));
    return RBFFD_OK;
}

static int op_array(const rbffd_plan* p, int32_t op, double** ptr, int64_t* count) {
    const OpBlock& b = (op == RBFFD_OP_CURL_E || op == RBFFD_OP_HV_E) ? p->opE : p->opH;
    if (op == RBFFD_OP_CURL_H || op == RBFFD_OP_CURL_E) {
        *ptr = b.wc;
        *count = b.Nt * p->dim * b.n;
    } else if (op == RBFFD_OP_HV_H || op == RBFFD_OP_HV_E) {
        *ptr = b.wh;
        *count = b.Nt * b.nh;
    } else {
        return set_err(p, RBFFD_EINVAL, "unknown operator selector");
    }
    if (!*ptr || *count == 0) return set_err(p, RBFFD_EINVAL, "operator not present in this plan");
    return RBFFD_OK;
}

extern "C" int rbffd_get_weights(const rbffd_plan* p, int32_t op, double* out, void* stream) {
    if (!p || !out) return RBFFD_EINVAL;
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    double* src;
    int64_t count;
    int rc = op_array(p, op, &src, &count);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(p, hipMemcpyAsync(out, src, count * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(p, hipStreamSynchronize(s));
    return RBFFD_OK;
}

extern "C" int rbffd_set_weights(rbffd_plan* p, int32_t op, const double* in, void* stream) {
    if (!p || !in) return RBFFD_EINVAL;
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    double* dst;
    int64_t count;
    int rc = op_array(p, op, &dst, &count);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(p, hipMemcpyAsync(dst, in, count * 8, hipMemcpyHostToDevice, s));
    rc = pack_all(p, nullptr, s);
    if (rc) return rc;
    if (p->p.adjoint && (rc = refill_transpose(p, s))) return rc;
    HIPCHK(p, hipStreamSynchronize(s));
    return RBFFD_OK;
}

extern "C" int rbffd_get_variant(const rbffd_plan* p, int32_t* v) {
    if (!p || !v) return RBFFD_EINVAL;
    *v = p->var.block | (p->var.xcd << 16) | (p->var.lds << 17) | (p->var.persist << 20);
    return RBFFD_OK;
}

extern "C" int rbffd_set_variant(rbffd_plan* p, int32_t block, int32_t xcd, int32_t lds, int32_t persist) {
    if (!p) return RBFFD_EINVAL;
    if (block < 64 || block > 512 || (block % 64) || persist < 1 || persist > 64 || lds < 0 || lds > 3)
        return set_err(p, RBFFD_EINVAL, "bad launch variant");
    p->var.block = block;
    p->var.xcd = xcd ? 1 : 0;
    p->var.lds = lds;
    p->var.persist = persist;
    return RBFFD_OK;
}
