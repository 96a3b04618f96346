// Set-up on the GPU: node ordering, exact kNN stencils, FP64 local weight
// systems, packing for the step kernels, transposed operators for the adjoint.
//
// Reference: Kolar-Pozun & Kosec (arXiv 2508.18205), Section 4 (eq. 8-15:
// stencils of the n nearest nodes, PHS + monomial interpolation systems,
// RBF-FD and RBF-VFD right-hand sides) and Section 5.1 (hyperviscosity by
// RBF-FD of Delta^alpha with phi = r^(2 alpha + 1), m = 2 alpha).  The paper
// computes the weights once before time stepping; so does this file.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "common.h"
#include "wpack.h"

namespace {

constexpr int MORTON_BITS_2D = 32;
constexpr int MORTON_BITS_3D = 21;

// ---------------------------------------------------------------------------
// Morton keys.  q_k = min(floor((x_k - lo_k) * scale), 2^b - 1), scale =
// 2^b / side computed once on the host (one correctly rounded division); key
// bit d*i + k = bit i of q_k.  Subtraction and multiplication are separate
// correctly rounded operations (no contraction possible), so keys are
// reproducible bit for bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t quantise(double x, double lo, double scale, int bits) {
    double q = floor((x - lo) * scale);
    if (q < 0.0) q = 0.0;
    uint64_t qi = (uint64_t)q;
    const uint64_t top = (1ull << bits) - 1ull;
    return qi > top ? top : qi;
}

__device__ __forceinline__ uint64_t interleave(const uint64_t* q, int d, int bits) {
    uint64_t key = 0;
    for (int i = 0; i < bits; ++i)
        for (int k = 0; k < d; ++k) key |= ((q[k] >> i) & 1ull) << (d * i + k);
    return key;
}

struct MortonArgs {
    const double* xyz;
    int64_t N;
    int d, bits;
    double lo[3];
    double scale;
    uint64_t* keys;
    int32_t* vals;
};

__global__ void k_morton(MortonArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    uint64_t q[3] = {0, 0, 0};
    for (int k = 0; k < a.d; ++k) q[k] = quantise(a.xyz[i * a.d + k], a.lo[k], a.scale, a.bits);
    a.keys[i] = interleave(q, a.d, a.bits);
    a.vals[i] = (int32_t)i;
}

// sorted coordinates and cell ranges of the search structure
__global__ void k_gather_sorted(const double* xyz, const int32_t* sperm, int64_t N, int d, double* sxyz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t o = sperm[i];
    for (int k = 0; k < d; ++k) sxyz[i * d + k] = xyz[(int64_t)o * d + k];
}

__global__ void k_cell_ranges(const uint64_t* skeys, int64_t N, int shift, int32_t* cstart, int32_t* cend) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint64_t c = skeys[i] >> shift;
    if (i == 0 || (skeys[i - 1] >> shift) != c) cstart[c] = (int32_t)i;
    if (i == N - 1 || (skeys[i + 1] >> shift) != c) cend[c] = (int32_t)(i + 1);
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_iota(int32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// Exact k nearest neighbours.  Key of candidate j for centre c: (d2, orig_j)
// with d2 = (dx*dx) + (dy*dy) [+ (dz*dz)], every product and sum rounded
// separately (contraction disabled below), so the order equals the oracle's.
// ---------------------------------------------------------------------------
struct KnnArgs {
    const double* cxyz;     // centres in iteration order [Nc][d]
    const int32_t* crow;    // output row of each centre
    int64_t Nc;
    const double* sxyz;     // sources sorted by Morton key [Ns][d]
    const int32_t* sorig;   // original id of each sorted source
    int64_t Ns;
    const int32_t* cstart;  // cell ranges (cells mode)
    const int32_t* cend;
    int d, k, L, bits;
    double lo[3];
    double scale, side;
    double period[3];       // periodic: axis lengths (domain [lo, lo + period))
    int periodic;
    int32_t* out;           // [rows][k] original source ids
};

__device__ __forceinline__ double sq_dist(const double* a, const double* b, int d, const double* per, int periodic) {
#pragma clang fp contract(off)
    double acc = 0.0;
    for (int k = 0; k < d; ++k) {
        double dk = b[k] - a[k];
        if (periodic) {
            const double L = per[k];
            if (dk > 0.5 * L) dk = dk - L;
            if (dk < -0.5 * L) dk = dk + L;
        }
        const double s = dk * dk;
        acc = (k == 0) ? s : acc + s;
    }
    return acc;
}

// The k smallest (d2, id) pairs seen so far, as a binary max-heap (the root is
// the current k-th nearest); finish() heap-sorts them into ascending order.
// Pairs are totally ordered (ids are distinct), so the result is the same
// list an insertion sort would give.
template <int KMAX>
struct TopK {
    double d2[KMAX];
    int32_t id[KMAX];
    int cnt = 0;
    __device__ static __forceinline__ bool gt(double a, int32_t ia, double b, int32_t ib) {
        return a > b || (a == b && ia > ib);
    }
    __device__ __forceinline__ void sift_down(double dd, int32_t o, int n) {
        int pos = 0;
        for (;;) {
            const int l = 2 * pos + 1;
            if (l >= n) break;
            const int r = l + 1;
            const int c = (r < n && gt(d2[r], id[r], d2[l], id[l])) ? r : l;
            if (!gt(d2[c], id[c], dd, o)) break;
            d2[pos] = d2[c];
            id[pos] = id[c];
            pos = c;
        }
        d2[pos] = dd;
        id[pos] = o;
    }
    __device__ __forceinline__ void push(double dd, int32_t o, int k) {
        if (cnt == k) {
            if (gt(dd, o, d2[0], id[0]) || (dd == d2[0] && o == id[0])) return;
            sift_down(dd, o, k);
            return;
        }
        int pos = cnt++;
        while (pos > 0) {
            const int par = (pos - 1) >> 1;
            if (!gt(dd, o, d2[par], id[par])) break;
            d2[pos] = d2[par];
            id[pos] = id[par];
            pos = par;
        }
        d2[pos] = dd;
        id[pos] = o;
    }
    // the current k-th smallest squared distance (valid once cnt == k)
    __device__ __forceinline__ double worst() const { return d2[0]; }
    __device__ __forceinline__ void finish() {
        for (int end = cnt - 1; end > 0; --end) {
            const double dd = d2[end];
            const int32_t o = id[end];
            d2[end] = d2[0];
            id[end] = id[0];
            sift_down(dd, o, end);
        }
    }
};

// Periodic image of source x seen from centre c: per axis -1, 0 or +1 as the
// wrapped difference of sq_dist takes L off, keeps, or adds L to x - c, packed
// base 3 (0 = no wrap).  Each source belongs to exactly one image of c.
__device__ __forceinline__ int wrap_code(const double* c, const double* x, int d, const double* per) {
    int code = 0, w = 1;
    for (int k = 0; k < d; ++k, w *= 3) {
        const double dk = x[k] - c[k];
        code += w * (dk > 0.5 * per[k] ? 2 : (dk < -0.5 * per[k] ? 1 : 0));
    }
    return code;
}

// Ring search of the cell grid around position q, cells in rings of growing
// Chebyshev radius, until every unscanned cell lies farther than the current
// k-th nearest.  Distances are taken from the centre c (periodic: wrapped);
// periodic searches keep only the sources of image `img` (q is that image of
// c, so the wrapped distance of such a source is its distance from q and the
// cell bounds hold for it).  Nodes outside the grid box sit in its edge cells,
// which only makes them farther than the bounds say.
template <int KMAX>
__device__ void ring_search(const KnnArgs& a, const double* c, const double* q, int img, TopK<KMAX>& tk) {
    const int G = 1 << a.L;
    const double cs = a.side / G;
    int cc[3] = {0, 0, 0};
    for (int k = 0; k < a.d; ++k) cc[k] = (int)(quantise(q[k], a.lo[k], a.scale, a.bits) >> (a.bits - a.L));
    for (int r = 0;; ++r) {
        const int z0 = a.d == 3 ? -r : 0, z1 = a.d == 3 ? r : 0;
        for (int dz = z0; dz <= z1; ++dz)
            for (int dy = -r; dy <= r; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    const int m = max(abs(dx), max(abs(dy), abs(dz)));
                    if (m != r) continue;
                    const int x = cc[0] + dx, y = cc[1] + dy, z = cc[2] + dz;
                    if (x < 0 || x >= G || y < 0 || y >= G || (a.d == 3 && (z < 0 || z >= G))) continue;
                    uint64_t qc[3] = {(uint64_t)x, (uint64_t)y, (uint64_t)z};
                    const uint64_t cid = interleave(qc, a.d, a.L);
                    const int32_t e = a.cend[cid];
                    for (int32_t j = a.cstart[cid]; j < e; ++j) {
                        const double* xs = a.sxyz + (int64_t)j * a.d;
                        if (a.periodic && wrap_code(c, xs, a.d, a.period) != img) continue;
                        tk.push(sq_dist(c, xs, a.d, a.period, a.periodic), a.sorig[j], a.k);
                    }
                }
        // every node outside the scanned box is at least R away
        bool whole = true;
        double R = 1e300;
        for (int k = 0; k < a.d; ++k) {
            if (cc[k] - r > 0) {
                whole = false;
                R = fmin(R, q[k] - (a.lo[k] + (cc[k] - r) * cs));
            }
            if (cc[k] + r < G - 1) {
                whole = false;
                R = fmin(R, (a.lo[k] + (cc[k] + r + 1) * cs) - q[k]);
            }
        }
        if (whole) break;
        R -= 1e-9 * cs;
        if (tk.cnt >= a.k && R > 0.0 && tk.worst() < R * R) break;
    }
}

// Periodic sets search the images c + s P (s in {-1, 0, 1}^d) of each centre,
// c itself first; an image farther from the domain box [lo, hi) (which holds
// every node of a periodic set) than the current k-th nearest holds none of
// the k nearest and is skipped.
template <int KMAX>
__global__ __launch_bounds__(64) void k_knn(KnnArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.Nc) return;
    double c[3] = {0, 0, 0};
    for (int k = 0; k < a.d; ++k) c[k] = a.cxyz[t * a.d + k];
    TopK<KMAX> tk;
    ring_search(a, c, c, 0, tk);
    if (a.periodic) {
        const int nimg = a.d == 3 ? 27 : 9;
        for (int img = 1; img < nimg; ++img) {
            double q[3] = {c[0], c[1], c[2]};
            double b2 = 0.0;
            for (int k = 0, v = img; k < a.d; ++k, v /= 3) {
                const int s = v % 3;   // 1: image c - L, 2: image c + L
                if (s == 1) q[k] = c[k] - a.period[k];
                if (s == 2) q[k] = c[k] + a.period[k];
                const double lo = a.lo[k], hi = a.lo[k] + a.period[k];
                const double g = q[k] < lo ? lo - q[k] : (q[k] > hi ? q[k] - hi : 0.0);
                b2 += g * g;
            }
            if (tk.cnt >= a.k && b2 * (1.0 - 1e-12) > tk.worst()) continue;
            ring_search(a, c, q, img, tk);
        }
    }
    tk.finish();
    const int64_t row = a.crow[t];
    for (int s = 0; s < a.k; ++s) a.out[row * a.k + s] = s < tk.cnt ? tk.id[s] : -1;
}

// relabel stencils of the target set into internal order
__global__ void k_relabel(const int32_t* knn_orig, int k, const int32_t* tperm, const int32_t* sinv, int64_t Nt,
                          int32_t* st, int width) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= Nt) return;
    const int64_t o = tperm[p];
    for (int s = 0; s < width; ++s) st[p * width + s] = sinv[knn_orig[o * k + s]];
}

__global__ void k_internal_nodes(const double* xyz_in, const uint8_t* flags_in, const int32_t* perm, int64_t N, int d,
                                 double* xyz, uint8_t* emask, int periodic, int te, const double* nrm_in,
                                 double* nrm) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t o = perm[p];
    for (int k = 0; k < d; ++k) xyz[p * d + k] = xyz_in[o * d + k];
    if (!emask) return;
    const uint8_t f = periodic ? 0 : flags_in[o];
    uint8_t keep;
    if (d == 2 && !te) {
        keep = f == 0 ? 1 : 0;              // Ez is tangential to every wall
    } else if (d == 2) {
        keep = 3;                           // (Ex, Ey): only the normal component survives
        for (int k = 0; k < 2; ++k)
            if (f & (3u << (2 * k))) keep &= (uint8_t)(1u << k);
        if (nrm) {                          // curved wall: project on the given normal
            const double nx = nrm_in[2 * o], ny = nrm_in[2 * o + 1];
            nrm[2 * p] = nx;
            nrm[2 * p + 1] = ny;
            if (nx != 0.0 || ny != 0.0) keep |= 8;
        }
    } else {
        keep = 7;
        for (int k = 0; k < 3; ++k)
            if (f & (3u << (2 * k))) keep &= (uint8_t)(1u << k);   // only the normal component survives
        if (nrm) {                          // curved wall: project on the given normal
            bool any = false;
            for (int k = 0; k < 3; ++k) {
                const double v = nrm_in[3 * o + k];
                nrm[3 * p + k] = v;
                any = any || v != 0.0;
            }
            if (any) keep |= 8;
        }
    }
    emask[p] = keep;
}

__global__ void k_inverse(const int32_t* perm, int64_t N, int32_t* inv) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) inv[perm[p]] = (int32_t)p;
}

// ---------------------------------------------------------------------------
// Local weight systems (eq. 9 with eq. 13 / eq. 15 right-hand sides; HV by
// RBF-FD of Delta^alpha).  One workgroup per centre, the augmented matrix
// [A~ | B] lives in LDS; Gaussian elimination with partial pivoting (largest
// |pivot|, lowest row on ties) and back substitution in FP64.
// ---------------------------------------------------------------------------
enum { W_FD = 0, W_VFD = 1, W_HV = 2 };

struct WArgs {
    const double* txyz;   // target centres (internal order) [Nt][d]
    const double* sxyz;   // source nodes (internal order) [Ns][d]
    const int32_t* st;    // stencil rows (internal labels of the source set)
    int st_stride;
    int n;                // stencil entries used
    int M;                // monomials
    int d;
    int kind;
    int phs_k;
    int nrhs;
    int upow;             // unscaling power l
    int periodic;
    double period[3];
    double vdelta;        // RBF-VFD virtual spacing (unscaled)
    double fu[3][3];      // derivative directions: right-hand side q acts along fu[q]
    double hv_C;          // Delta^alpha r^(2a+1) = hv_C r
    double hv_poly[RBFFD_MAX_MONO];
    int8_t ex[RBFFD_MAX_MONO][3];
    double* out;          // [Nt][nrhs][n]
    int64_t Nt;
    int64_t c0;           // first centre of this launch
    int32_t* status;      // status[0] = first singular centre (atomicMin), status[1] = self-first violations
    int check_self;
};

__device__ __forceinline__ double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

__device__ __forceinline__ double phs(double r, int k) {
    // r^k for odd k >= 3
    double r2 = r * r;
    double v = r;
    for (int i = 0; i < (k - 1) / 2; ++i) v *= r2;
    return v;
}

__device__ __forceinline__ double mono(const double* x, const int8_t* e, int d) {
    double v = 1.0;
    for (int k = 0; k < d; ++k) v *= ipow(x[k], e[k]);
    return v;
}

// u . grad p at 0 for the monomial with exponents e: u_k for p = x_k, else 0
__device__ __forceinline__ double dmono_at0(const int8_t* e, int d, const double* u) {
    int deg = 0, ax = 0;
    for (int k = 0; k < d; ++k) {
        deg += e[k];
        if (e[k] == 1) ax = k;
    }
    return deg == 1 ? u[ax] : 0.0;
}

// Entry (i, j) of the augmented local system [A~ | B] (eq. 9 with the
// eq. 13 / eq. 15 / Delta^alpha right-hand sides) from the scaled offsets xi
// [n][3] and the stencil scale sc.
__device__ __forceinline__ double system_entry(const WArgs& a, const double* xi, double sc, int i, int j) {
    const int n = a.n, R = n + a.M, d = a.d;
    double v = 0.0;
    if (j < R) {
        if (i < n && j < n) {
            double r2 = 0.0;
            for (int k = 0; k < d; ++k) {
                const double t = xi[i * 3 + k] - xi[j * 3 + k];
                r2 += t * t;
            }
            v = phs(sqrt(r2), a.phs_k);
        } else if (i < n && j >= n) {
            v = mono(xi + i * 3, a.ex[j - n], d);
        } else if (i >= n && j < n) {
            v = mono(xi + j * 3, a.ex[i - n], d);
        }
    } else {
        const int col = j - R;   // right-hand side index (derivative direction)
        const double* u = a.fu[col];
        if (a.kind == W_FD) {
            if (i < n) {
                double r2 = 0.0, xu = 0.0;
                for (int k = 0; k < d; ++k) {
                    r2 += xi[i * 3 + k] * xi[i * 3 + k];
                    xu += xi[i * 3 + k] * u[k];
                }
                const double r = sqrt(r2);
                // u . grad |x - xi_i|^k at x = 0 = -k r^(k-2) (xi_i . u)
                v = -(double)a.phs_k * phs(r, a.phs_k - 2) * xu;
            } else {
                v = dmono_at0(a.ex[i - n], d, u);
            }
        } else if (a.kind == W_VFD) {
            // central virtual difference: (-1/2 f(-delta u) + 1/2 f(+delta u)) / delta
            const double dl = a.vdelta / sc;
            double xm[3] = {0, 0, 0}, xp[3] = {0, 0, 0};
            for (int k = 0; k < d; ++k) {
                xm[k] = -dl * u[k];
                xp[k] = dl * u[k];
            }
            double fm, fp;
            if (i < n) {
                double r2m = 0.0, r2p = 0.0;
                for (int k = 0; k < d; ++k) {
                    const double tm = xm[k] - xi[i * 3 + k], tp = xp[k] - xi[i * 3 + k];
                    r2m += tm * tm;
                    r2p += tp * tp;
                }
                fm = phs(sqrt(r2m), a.phs_k);
                fp = phs(sqrt(r2p), a.phs_k);
            } else {
                fm = mono(xm, a.ex[i - n], d);
                fp = mono(xp, a.ex[i - n], d);
            }
            v = (-0.5 * fm + 0.5 * fp) / dl;
        } else {
            if (i < n) {
                double r2 = 0.0;
                for (int k = 0; k < d; ++k) r2 += xi[i * 3 + k] * xi[i * 3 + k];
                v = a.hv_C * sqrt(r2);
            } else {
                v = a.hv_poly[i - n];
            }
        }
    }
    return v;
}

// A pivot no larger than 1024 R eps max_ij |A~_ij| (R unknowns, eps the FP64
// machine epsilon, A~ the scaled system before elimination) marks the local
// system as numerically singular: every valid stencil of the benchmarked node
// sets keeps its pivots above ~1e8 R eps max|A~| (condition numbers up to
// ~1e7), while collinear stencils and nodes closer than ~1e-11 h fall below.
__device__ __forceinline__ double pivot_floor(int R, double amax) {
    return 1024.0 * (double)R * 2.220446049250313e-16 * amax;
}

__global__ __launch_bounds__(1024) void k_weights(WArgs a) {
    extern __shared__ double lds[];
    const int64_t c = a.c0 + blockIdx.x;
    if (c >= a.Nt) return;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int n = a.n, M = a.M, R = n + M, d = a.d;
    const int lda = R + a.nrhs;
    double* Am = lds;                        // [R][lda]
    double* xi = Am + R * lda;               // [n][3]
    double* piv = xi + n * 3;                // [R] multipliers
    __shared__ double s_scale;
    __shared__ int s_p;
    __shared__ int s_bad;

    // 1. offsets from the centre and the stencil radius
    const double* xc = a.txyz + c * d;
    const int32_t* row = a.st + c * a.st_stride;
    for (int j = tid; j < n; j += nt) {
        const double* xj = a.sxyz + (int64_t)row[j] * d;
        for (int k = 0; k < 3; ++k) xi[j * 3 + k] = 0.0;
        for (int k = 0; k < d; ++k) {
            double dk = xj[k] - xc[k];
            if (a.periodic) {
                const double L = a.period[k];
                if (dk > 0.5 * L) dk -= L;
                if (dk < -0.5 * L) dk += L;
            }
            xi[j * 3 + k] = dk;
        }
    }
    if (tid == 0) {
        s_bad = 0;
        if (a.check_self && row[0] != (int32_t)c) atomicAdd(&a.status[1], 1);
    }
    __syncthreads();
    if (tid < 64) {
        double mx = 0.0;
        for (int j = tid; j < n; j += 64) {
            double r2 = 0.0;
            for (int k = 0; k < d; ++k) r2 += xi[j * 3 + k] * xi[j * 3 + k];
            mx = fmax(mx, sqrt(r2));
        }
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
        if (tid == 0) s_scale = mx;
    }
    __syncthreads();
    const double sc = s_scale;
    for (int j = tid; j < n * 3; j += nt) xi[j] = xi[j] / sc;
    __syncthreads();

    // 2. assemble [A~ | B]
    for (int e = tid; e < R * lda; e += nt) {
        const int i = e / lda, j = e % lda;
        const double v = system_entry(a, xi, sc, i, j);
        Am[i * lda + j] = v;
    }
    __syncthreads();
    // singularity threshold relative to the scaled system's largest entry
    __shared__ double s_tau;
    if (tid < 64) {
        double mx = 0.0;
        for (int e = tid; e < R * R; e += 64) mx = fmax(mx, fabs(Am[(e / R) * lda + e % R]));
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
        if (tid == 0) s_tau = pivot_floor(R, mx);
    }
    __syncthreads();
    const double tau = s_tau;

    // 3. forward elimination with partial pivoting.  Rows are addressed
    // through prm (logical row -> row of Am), so a pivot exchange is a swap of
    // two entries; wavefront 0 picks the pivot (largest |value| in column k,
    // ties to the lower logical row) and computes the multipliers, then every
    // thread updates the trailing block: two barriers per column.
    __shared__ int prm[RBFFD_MAX_STENCIL + RBFFD_MAX_MONO];
    for (int i = tid; i < R; i += nt) prm[i] = i;
    __syncthreads();
    for (int k = 0; k < R; ++k) {
        if (tid < 64) {
            double best = -1.0;
            int bi = R;
            for (int i = k + tid; i < R; i += 64) {
                const double v = fabs(Am[prm[i] * lda + k]);
                if (v > best) { best = v; bi = i; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ob = __shfl_xor(best, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            // every lane now holds the pivot's logical row bi
            const int rk = prm[k], rp = prm[bi];
            if (!(best > tau)) {
                if (tid == 0) s_bad = 1;
            } else {
                const double pk = Am[rp * lda + k];
                // after the exchange logical row bi holds the old row k
                for (int i = k + 1 + tid; i < R; i += 64) {
                    const int ri = (i == bi) ? rk : prm[i];
                    piv[i] = Am[ri * lda + k] / pk;
                }
            }
            if (tid == 0) {
                prm[bi] = rk;
                prm[k] = rp;
            }
        }
        __syncthreads();
        if (s_bad) break;
        const int rk = prm[k];
        const int rows = R - k - 1, cols = lda - k - 1;
        for (int e = tid; e < rows * cols; e += nt) {
            const int i = k + 1 + e / cols, j = k + 1 + e % cols;
            Am[prm[i] * lda + j] -= piv[i] * Am[rk * lda + j];
        }
        __syncthreads();
    }
    if (s_bad) {
        if (tid == 0) atomicMin(&a.status[0], (int32_t)c);
        for (int e = tid; e < a.nrhs * n; e += nt) a.out[c * a.nrhs * n + e] = 0.0;
        return;
    }
    // 4. back substitution, column by column of the unknowns
    for (int i = R - 1; i >= 0; --i) {
        const int ri = prm[i];
        const double di = Am[ri * lda + i];
        for (int q = tid; q < a.nrhs; q += nt) Am[ri * lda + R + q] /= di;
        __syncthreads();
        for (int e = tid; e < i * a.nrhs; e += nt) {
            const int r = prm[e / a.nrhs], q = e % a.nrhs;
            Am[r * lda + R + q] -= Am[r * lda + i] * Am[ri * lda + R + q];
        }
        __syncthreads();
    }
    // 5. unscale and store the first n entries (unknown j sits in row prm[j])
    const double us = ipow(sc, a.upow);
    for (int e = tid; e < a.nrhs * n; e += nt) {
        const int q = e / n, j = e % n;
        a.out[c * a.nrhs * n + e] = Am[prm[j] * lda + R + q] / us;
    }
}

// Register-resident variant for systems with R + nrhs <= 16 B (B <= 7): a
// 256-thread workgroup per system seen as a 16 x 16 grid; thread (tr, tc)
// holds the entries (tr + 16 a, tc + 16 b), a, b < B, of [A~ | B] in
// registers.  Gauss-Jordan elimination with partial pivoting (largest |value|
// among the rows not yet used as pivots, ties to the lower row): one barrier
// after the pivot candidates, one after the pivot row and the multipliers are
// published in LDS, per column; no back substitution.  The LDS footprint is
// ~20 KB (mostly the assembly band), so registers, not LDS, set how many
// systems share a CU (the LDS-resident kernel holds one 106-unknown system
// per CU).
constexpr int WREG_T = 16, WREG_BMAX = 7, WREG_MAX = WREG_T * WREG_BMAX;

// Column b / row r of the register block for an index that is the same in
// every thread: a switch on it compiles to scalar branches, and each case
// reads the registers with compile-time indices.
template <int B>
__device__ __forceinline__ void reg_col(const double (&m)[B][B], int b, double (&out)[B]) {
    switch (b) {
#define WREG_COL(C)                                                            \
    case C:                                                                    \
        _Pragma("unroll") for (int r = 0; r < B; ++r) out[r] = m[r][C < B ? C : B - 1]; \
        break;
        WREG_COL(0) WREG_COL(1) WREG_COL(2) WREG_COL(3) WREG_COL(4) WREG_COL(5)
#undef WREG_COL
        default:
            _Pragma("unroll") for (int r = 0; r < B; ++r) out[r] = m[r][B - 1];
    }
}
template <int B>
__device__ __forceinline__ void reg_row(const double (&m)[B][B], int a, double (&out)[B]) {
    switch (a) {
#define WREG_ROW(A)                                                            \
    case A:                                                                    \
        _Pragma("unroll") for (int q = 0; q < B; ++q) out[q] = m[A < B ? A : B - 1][q]; \
        break;
        WREG_ROW(0) WREG_ROW(1) WREG_ROW(2) WREG_ROW(3) WREG_ROW(4) WREG_ROW(5)
#undef WREG_ROW
        default:
            _Pragma("unroll") for (int q = 0; q < B; ++q) out[q] = m[B - 1][q];
    }
}

template <int WREG_B>
__global__ __launch_bounds__(256, 3) void k_wreg(WArgs a) {
    __shared__ double xi[WREG_MAX * 3];
    __shared__ double band[WREG_T * WREG_MAX];   // one 16-row band during assembly
    __shared__ double prow[WREG_MAX], mcol[WREG_MAX], dpiv[WREG_MAX];
    __shared__ double cval[WREG_T];              // [0]: the pivot candidate of column k
    __shared__ int cidx[WREG_T];
    __shared__ int kof[WREG_MAX];                // column pivoted on row i, -1 before
    __shared__ double s_scale;
    const int64_t c = a.c0 + blockIdx.x;
    if (c >= a.Nt) return;                       // uniform over the workgroup
    // thread (tr, tc): the 16 threads of one register column tc are 16
    // consecutive lanes of one wavefront, so the column steps of the
    // elimination run in a single wavefront
    const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
    const int n = a.n, R = n + a.M, d = a.d;
    const int lda = R + a.nrhs;

    // 1. offsets from the centre and the stencil radius (as k_weights)
    const double* xc = a.txyz + c * d;
    const int32_t* row = a.st + c * a.st_stride;
    for (int j = tid; j < n; j += 256) {
        const double* xj = a.sxyz + (int64_t)row[j] * d;
        for (int k = 0; k < 3; ++k) xi[j * 3 + k] = 0.0;
        for (int k = 0; k < d; ++k) {
            double dk = xj[k] - xc[k];
            if (a.periodic) {
                const double L = a.period[k];
                if (dk > 0.5 * L) dk -= L;
                if (dk < -0.5 * L) dk += L;
            }
            xi[j * 3 + k] = dk;
        }
    }
    for (int i = tid; i < WREG_MAX; i += 256) {
        kof[i] = -1;
        prow[i] = 0.0;
        mcol[i] = 0.0;
    }
    if (tid == 0 && a.check_self && row[0] != (int32_t)c) atomicAdd(&a.status[1], 1);
    __syncthreads();
    if (tid < 64) {
        double mx = 0.0;
        for (int j = tid; j < n; j += 64) {
            double r2 = 0.0;
            for (int k = 0; k < d; ++k) r2 += xi[j * 3 + k] * xi[j * 3 + k];
            mx = fmax(mx, sqrt(r2));
        }
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
        if (tid == 0) s_scale = mx;
    }
    __syncthreads();
    const double sc = s_scale;
    for (int j = tid; j < n * 3; j += 256) xi[j] = xi[j] / sc;
    __syncthreads();

    // 2. assemble band by band through LDS into the registers
    double m[WREG_B][WREG_B];
#pragma unroll
    for (int ra = 0; ra < WREG_B; ++ra) {
        for (int e = tid; e < WREG_T * lda; e += 256) {
            const int i = WREG_T * ra + e / lda, j = e % lda;
            band[e] = i < R ? system_entry(a, xi, sc, i, j) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int cb = 0; cb < WREG_B; ++cb) {
            const int j = tc + WREG_T * cb;
            m[ra][cb] = j < lda ? band[tr * lda + j] : 0.0;
        }
        __syncthreads();
    }

    // singularity threshold relative to the largest entry of the square
    // system: a wavefront maximum, then the four wavefronts' through LDS
    double tau;
    {
        double mx = 0.0;
#pragma unroll
        for (int ra = 0; ra < WREG_B; ++ra)
#pragma unroll
            for (int cb = 0; cb < WREG_B; ++cb) {
                const bool in = (tr + WREG_T * ra < R) & (tc + WREG_T * cb < R);
                mx = in ? fmax(mx, fabs(m[ra][cb])) : mx;
            }
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
        if ((tid & 63) == 0) cval[tid >> 6] = mx;
        __syncthreads();
        tau = pivot_floor(R, fmax(fmax(cval[0], cval[1]), fmax(cval[2], cval[3])));
        __syncthreads();                         // cval is reused by the pivot search
    }
    // 3. Gauss-Jordan elimination.  The padding rows (i >= R) and columns
    // (j >= lda) hold zeros and stay zero, so every step below is written
    // without per-element branches: predicates become selects and LDS reads
    // are unconditional (all arrays have WREG_MAX entries).
    bool bad = false;
    for (int k = 0; k < R; ++k) {
        const int bk = k >> 4, ck = k & 15;
        if ((tid >> 6) == (ck >> 2)) {           // the wavefront holding column k
            double best = -1.0, bval = 0.0;
            int bi = R;
            if (tc == ck) {
                double colk[WREG_B];
                reg_col(m, bk, colk);
#pragma unroll
                for (int ra = 0; ra < WREG_B; ++ra) {
                    const int i = tr + WREG_T * ra;
                    const double v = colk[ra];
                    const bool take = (i < R) & (kof[i] < 0) & (fabs(v) > best);
                    best = take ? fabs(v) : best;
                    bval = take ? v : bval;
                    bi = take ? i : bi;
                }
            }
            // reduce over the 16 lanes of each column (lanes 16 q .. 16 q + 15)
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const double ob = __shfl_xor(best, off, 64), ov = __shfl_xor(bval, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                const bool take = (ob > best) | ((ob == best) & (oi < bi));
                best = take ? ob : best;
                bval = take ? ov : bval;
                bi = take ? oi : bi;
            }
            if (tid == (ck << 4)) {               // tr = 0 of column ck
                cval[0] = bval;
                cidx[0] = bi;
            }
        }
        __syncthreads();
        const int p = cidx[0];
        const double pval = cval[0], pbest = p < R ? fabs(pval) : -1.0;
        if (!(pbest > tau)) {                    // the same decision in every thread
            bad = true;
            break;
        }
        if (tr == (p & 15)) {
            double rowp[WREG_B];
            reg_row(m, p >> 4, rowp);
#pragma unroll
            for (int cb = 0; cb < WREG_B; ++cb) prow[tc + WREG_T * cb] = rowp[cb];
        }
        if (tc == ck) {
            double colk[WREG_B];
            reg_col(m, bk, colk);
            const double rp = 1.0 / pval;
#pragma unroll
            for (int ra = 0; ra < WREG_B; ++ra) {
                const int i = tr + WREG_T * ra;
                mcol[i] = (i == p) ? 0.0 : colk[ra] * rp;
            }
        }
        if (tid == 0) {
            kof[p] = k;
            dpiv[k] = pval;
        }
        __syncthreads();
        double pj[WREG_B];
#pragma unroll
        for (int cb = 0; cb < WREG_B; ++cb) {
            const int j = tc + WREG_T * cb;
            pj[cb] = (j > k) ? prow[j] : 0.0;
        }
#pragma unroll
        for (int ra = 0; ra < WREG_B; ++ra) {
            const double mi = mcol[tr + WREG_T * ra];
#pragma unroll
            for (int cb = 0; cb < WREG_B; ++cb) m[ra][cb] -= mi * pj[cb];
        }
    }
    if (bad) {
        if (tid == 0) atomicMin(&a.status[0], (int32_t)c);
        for (int e = tid; e < a.nrhs * n; e += 256) a.out[c * a.nrhs * n + e] = 0.0;
        return;
    }
    // 4. unknown k sits in the row pivoted at column k; unscale and store the
    // first n entries of every right-hand side
    const double us = ipow(sc, a.upow);
#pragma unroll
    for (int ra = 0; ra < WREG_B; ++ra) {
        const int i = tr + WREG_T * ra;
        if (i >= R) continue;
        const int k = kof[i];
        if (k >= n) continue;
#pragma unroll
        for (int cb = 0; cb < WREG_B; ++cb) {
            const int j = tc + WREG_T * cb;
            if (j >= R && j < lda) a.out[c * a.nrhs * n + (int64_t)(j - R) * n + k] = m[ra][cb] / dpiv[k] / us;
        }
    }
}

// ---------------------------------------------------------------------------
// Packing for the step kernels
// ---------------------------------------------------------------------------
template <typename TW>
__global__ void k_pack_union(const int32_t* st, const double* wc, const double* wh, int64_t N, int ns, int n, int nh,
                             int d, int C4, int V4, int S4, int64_t tiles, int4* pidx, TW* pwc, TW* pwh) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (tile, lane)
    if (g >= tiles * RBFFD_TILE) return;
    const int64_t tile = g / RBFFD_TILE;
    const int lane = (int)(g % RBFFD_TILE);
    const int64_t i = g;
    const bool real = i < N;
    const int64_t ic = real ? i : N - 1;
    for (int q = 0; q < S4; ++q) {
        int v[4];
        for (int u = 0; u < 4; ++u) {
            const int s = 1 + 4 * q + u;
            v[u] = (real && s < ns) ? st[ic * ns + s] : (int)ic;
        }
        pidx[(tile * S4 + q) * RBFFD_TILE + lane] = make_int4(v[0], v[1], v[2], v[3]);
    }
    for (int q = 0; q < C4; ++q)
        for (int ax = 0; ax < d; ++ax) {
            double w[4];
            for (int u = 0; u < 4; ++u) {
                const int s = 1 + 4 * q + u;
                w[u] = (real && s < n) ? wc[(ic * d + ax) * n + s] : 0.0;
            }
            WF<TW>::store(pwc + ((tile * C4 + q) * d + ax) * WF<TW>::CH + lane * WF<TW>::LS, w);
        }
    for (int q = 0; q < V4; ++q) {
        double w[4];
        for (int u = 0; u < 4; ++u) {
            const int s = 1 + 4 * q + u;
            w[u] = (real && s < nh) ? wh[ic * nh + s] : 0.0;
        }
        WF<TW>::store(pwh + (tile * V4 + q) * WF<TW>::CH + lane * WF<TW>::LS, w);
    }
}

template <typename TW>
__global__ void k_pack_cross(const int32_t* stc, const int32_t* sth, const double* wc, const double* wh, int64_t N,
                             int n, int nh, int d, int C4, int V4, int64_t tiles, int4* pidx, int4* pidx_h,
                             int32_t* pref, TW* pwc, TW* pwh) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= tiles * RBFFD_TILE) return;
    const int64_t tile = g / RBFFD_TILE;
    const int lane = (int)(g % RBFFD_TILE);
    const bool real = g < N;
    const int64_t ic = real ? g : N - 1;
    const int ref = stc[ic * n];
    if (real) pref[g] = ref;
    for (int q = 0; q < C4; ++q) {
        int v[4];
        for (int u = 0; u < 4; ++u) {
            const int s = 1 + 4 * q + u;
            v[u] = (real && s < n) ? stc[ic * n + s] : ref;
        }
        pidx[(tile * C4 + q) * RBFFD_TILE + lane] = make_int4(v[0], v[1], v[2], v[3]);
        for (int ax = 0; ax < d; ++ax)
            for (int u = 0; u < 4; ++u) {
                const int s = 1 + 4 * q + u;
                const double w = (real && s < n) ? wc[(ic * d + ax) * n + s] : 0.0;
                pwc[((tile * C4 + q) * d + ax) * RBFFD_TILE * 4 + WChunk<TW>::at(lane, u)] = (TW)w;
            }
    }
    for (int q = 0; q < V4; ++q) {
        int v[4];
        for (int u = 0; u < 4; ++u) {
            const int s = 1 + 4 * q + u;
            v[u] = (real && s < nh) ? sth[ic * nh + s] : (int)ic;
            const double w = (real && s < nh) ? wh[ic * nh + s] : 0.0;
            pwh[(tile * V4 + q) * RBFFD_TILE * 4 + WChunk<TW>::at(lane, u)] = (TW)w;
        }
        pidx_h[(tile * V4 + q) * RBFFD_TILE + lane] = make_int4(v[0], v[1], v[2], v[3]);
    }
}

// K-field batch (2D): the neighbour slots as in the union pack, plus the
// centre weights of the curl and hyperviscosity operators in FP32 (the batch
// kernels sum eq. 16 over the whole stencil, centre included)
__global__ void k_pack_batched(const int32_t* st, const double* wc, const double* wh, int64_t N, int ns, int n, int nh,
                               int d, int C4, int V4, int S4, int32_t* bidx, float* bwc, float* bwh, float* bw0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    bw0[i * 4 + 0] = (float)wc[(i * d + 0) * n];
    bw0[i * 4 + 1] = d > 1 ? (float)wc[(i * d + 1) * n] : 0.0f;
    bw0[i * 4 + 2] = nh > 0 ? (float)wh[i * nh] : 0.0f;
    bw0[i * 4 + 3] = 0.0f;
    for (int s4 = 0; s4 < S4 * 4; ++s4) {
        const int s = 1 + s4;
        bidx[i * S4 * 4 + s4] = s < ns ? st[i * ns + s] : (int)i;
    }
    for (int ax = 0; ax < d; ++ax)
        for (int s4 = 0; s4 < C4 * 4; ++s4) {
            const int s = 1 + s4;
            bwc[(i * d + ax) * C4 * 4 + s4] = s < n ? (float)wc[(i * d + ax) * n + s] : 0.0f;
        }
    for (int s4 = 0; s4 < V4 * 4; ++s4) {
        const int s = 1 + s4;
        bwh[i * V4 * 4 + s4] = s < nh ? (float)wh[i * nh + s] : 0.0f;
    }
}

// ---------------------------------------------------------------------------
// Transposed operator (adjoint): entries (j <- i, slot s) sorted by (j, i, s)
// ---------------------------------------------------------------------------
__global__ void k_tkeys(const int32_t* st, int64_t N, int ns, uint64_t* keys) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N * ns) return;
    const int64_t i = e / ns;
    const int s = (int)(e % ns);
    const uint64_t j = (uint64_t)st[e];
    keys[e] = j * (uint64_t)(N * ns) + (uint64_t)(i * ns + s);
}

__global__ void k_tdeg(const uint64_t* skeys, int64_t E, int64_t Nns, int32_t* rstart, int32_t* rend) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int64_t j = (int64_t)(skeys[e] / (uint64_t)Nns);
    if (e == 0 || (int64_t)(skeys[e - 1] / (uint64_t)Nns) != j) rstart[j] = (int32_t)e;
    if (e == E - 1 || (int64_t)(skeys[e + 1] / (uint64_t)Nns) != j) rend[j] = (int32_t)(e + 1);
}

__global__ void k_twidth(const int32_t* rstart, const int32_t* rend, int64_t N, int64_t tiles, int32_t* width) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tiles) return;
    int w = 0;
    for (int l = 0; l < RBFFD_TILE; ++l) {
        const int64_t j = t * RBFFD_TILE + l;
        if (j < N) w = max(w, rend[j] - rstart[j]);
    }
    width[t] = w;
}

// SELL layout of D^T: entry (tile t, column q, lane l) = the q-th incoming
// entry of row j = 64 t + l; records the source row i and the slot s
__global__ void k_tfill(const uint64_t* skeys, const int32_t* rstart, const int32_t* rend, const int64_t* toff,
                        const int32_t* width, int64_t N, int ns, int64_t tiles, int32_t* tsrc, int32_t* tslot) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= tiles * RBFFD_TILE) return;
    const int64_t t = g / RBFFD_TILE;
    const int l = (int)(g % RBFFD_TILE);
    const int64_t j = g;
    const int w = width[t];
    const int deg = j < N ? rend[j] - rstart[j] : 0;
    const int64_t jc = j < N ? j : N - 1;
    for (int q = 0; q < w; ++q) {
        const int64_t e = toff[t] + (int64_t)q * RBFFD_TILE + l;
        if (q < deg) {
            const uint64_t key = skeys[rstart[j] + q];
            const int64_t rem = (int64_t)(key % (uint64_t)(N * ns));
            tsrc[e] = (int32_t)(rem / ns);
            tslot[e] = (int32_t)(rem % ns);
        } else {
            tsrc[e] = (int32_t)jc;
            tslot[e] = -1;
        }
    }
}

// transposed weights (wx, wy, wh, 0) of every SELL entry from the FP64 weights
template <typename TW>
// the transposed weights of each entry, one array per operator ([3][cap]:
// D^dx, D^dy, D^hv) so that a wavefront's load of one of them is contiguous
__global__ void k_tweights(const int32_t* tsrc, const int32_t* tslot, int64_t E, const double* wc, const double* wh,
                           int n, int nh, int64_t cap, TW* tw) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int s = tslot[e];
    const int64_t i = tsrc[e];
    tw[e] = (TW)((s >= 0 && s < n) ? wc[(i * 2 + 0) * n + s] : 0.0);
    tw[cap + e] = (TW)((s >= 0 && s < n) ? wc[(i * 2 + 1) * n + s] : 0.0);
    tw[2 * cap + e] = (TW)((s >= 0 && s < nh) ? wh[i * nh + s] : 0.0);
}

// ---------------------------------------------------------------------------
// Halo lists for LDS staging: per workgroup tile (256 nodes in 2D; in 3D 1024
// with FP32 weights, 512 with FP64; 128 in K-field batch plans) the sorted
// unique source nodes of its
// stencils, and per (node, slot) the 16-bit position of the slot's node in
// that list.  Built from one global sort of (tile, source) keys.
// ---------------------------------------------------------------------------
__global__ void k_hkeys(const int32_t* st, int64_t N, int ns, int tsz, uint64_t* keys) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N * ns) return;
    const int64_t i = e / ns;
    keys[e] = ((uint64_t)(i / tsz) << 32) | (uint64_t)(uint32_t)st[e];
}

__global__ void k_hflags(const uint64_t* sk, int64_t E, int32_t* flag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < E) flag[e] = (e == 0 || sk[e] != sk[e - 1]) ? 1 : 0;
}

__global__ void k_hcompact(const uint64_t* sk, const int32_t* flag, const int32_t* pos, int64_t E, int32_t* pool,
                           int32_t* hoff, int64_t nwg) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    if (flag[e]) {
        pool[pos[e]] = (int32_t)(sk[e] & 0xFFFFFFFFull);
        const uint64_t t = sk[e] >> 32;
        if (e == 0 || (sk[e - 1] >> 32) != t) hoff[t] = pos[e];
    }
    if (e == E - 1) hoff[nwg] = pos[e] + flag[e];
}

__device__ __forceinline__ int lower_pos(const int32_t* a, int n, int32_t v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void k_hlocal(const int32_t* st, int64_t N, int ns, const int32_t* pool, const int32_t* hoff, int Q8,
                         int64_t tiles, int tsz, uint16_t* lidx, uint16_t* lself) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= tiles * RBFFD_TILE) return;
    const int64_t tile = g / RBFFD_TILE;
    const int lane = (int)(g % RBFFD_TILE);
    const bool real = g < N;
    const int64_t wg = g / tsz;
    const int32_t* L = pool + hoff[wg];
    const int cnt = hoff[wg + 1] - hoff[wg];
    const int self = real ? lower_pos(L, cnt, (int32_t)g) : 0;
    if (lself) lself[g] = (uint16_t)self;
    for (int q = 0; q < Q8; ++q)
        for (int u = 0; u < 8; ++u) {
            const int s = 1 + 8 * q + u;
            const int pos = (real && s < ns) ? lower_pos(L, cnt, st[g * ns + s]) : self;
            lidx[((tile * Q8 + q) * RBFFD_TILE + lane) * 8 + u] = (uint16_t)pos;
        }
}

// ---------------------------------------------------------------------------
// workspace bump allocator
// ---------------------------------------------------------------------------
struct WS {
    char* base;
    int64_t off = 0;
    template <typename T>
    T* take(int64_t count) {
        off = align_up(off, 256);
        T* r = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * (int64_t)sizeof(T);
        return r;
    }
};

inline int blocks(int64_t n, int b = 256) { return (int)cdiv(n, b); }

int cell_level(int64_t N, int d, int width) {
    const double target = std::max(8.0, width * 0.5);
    const double cells = std::max(1.0, (double)N / target);
    int L = (int)std::lround(std::log2(cells) / d);
    const int maxL = d == 2 ? 11 : 7;
    return std::max(1, std::min(L, maxL));
}

// Temporary storage of the radix sorts.  The query needs no device memory;
// should it fail (no device visible) a generous bound is used instead, which
// only matters for sizes reported before any GPU work.
size_t sort_temp_bytes(int64_t N) {
    size_t t = 0;
    if (rocprim::radix_sort_pairs(nullptr, t, (uint64_t*)nullptr, (uint64_t*)nullptr, (int32_t*)nullptr,
                                  (int32_t*)nullptr, (int)N, 0, 64) != hipSuccess)
        t = (size_t)N * 24 + (1u << 22);
    return t;
}

size_t scan_temp_bytes(int64_t E) {
    size_t t = 0;
    if (rocprim::exclusive_scan(nullptr, t, (int32_t*)nullptr, (int32_t*)nullptr, (int32_t)0, (size_t)E,
                                rocprim::plus<int32_t>()) != hipSuccess)
        t = (size_t)E / 64 + (1u << 22);
    return t;
}

size_t key_sort_temp_bytes(int64_t E) {
    size_t t = 0;
    if (rocprim::radix_sort_keys(nullptr, t, (uint64_t*)nullptr, (uint64_t*)nullptr, (int)E, 0, 64) != hipSuccess)
        t = (size_t)E * 16 + (1u << 22);
    return t;
}

// Search structure of one node set inside the workspace
struct Search {
    uint64_t* keys_in;
    uint64_t* keys;
    int32_t* vals_in;
    int32_t* sperm;     // sorted position -> original id
    double* sxyz;       // sorted coordinates
    int32_t* cstart;
    int32_t* cend;
    void* temp;
    size_t temp_bytes;
    int L;
    int64_t ncells;
};

void take_search(WS& w, Search& s, int64_t N, int d, int width, bool periodic) {
    s.keys_in = w.take<uint64_t>(N);
    s.keys = w.take<uint64_t>(N);
    s.vals_in = w.take<int32_t>(N);
    s.sperm = w.take<int32_t>(N);
    s.sxyz = w.take<double>(N * d);
    s.L = cell_level(N, d, width);
    s.ncells = (int64_t)1 << (d * s.L);
    s.cstart = w.take<int32_t>(s.ncells);
    s.cend = w.take<int32_t>(s.ncells);
    s.temp_bytes = sort_temp_bytes(N);
    s.temp = w.take<char>((int64_t)s.temp_bytes);
}

int build_search(rbffd_plan* p, NodeSet& S, Search& s, hipStream_t st) {
    const int d = p->dim;
    const int bits = d == 2 ? MORTON_BITS_2D : MORTON_BITS_3D;
    MortonArgs ma{};
    ma.xyz = S.xyz_in;
    ma.N = S.N;
    ma.d = d;
    ma.bits = bits;
    for (int k = 0; k < 3; ++k) ma.lo[k] = p->mlo[k];
    ma.scale = std::ldexp(1.0, bits) / p->mside;
    ma.keys = s.keys_in;
    ma.vals = s.vals_in;
    hipLaunchKernelGGL(k_morton, dim3(blocks(S.N)), dim3(256), 0, st, ma);
    size_t tb = s.temp_bytes;
    HIPCHK(p, rocprim::radix_sort_pairs(s.temp, tb, s.keys_in, s.keys, s.vals_in, s.sperm, (int)S.N, 0,
                                        (unsigned)(d * bits), st));
    hipLaunchKernelGGL(k_gather_sorted, dim3(blocks(S.N)), dim3(256), 0, st, S.xyz_in, s.sperm, S.N, d, s.sxyz);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(s.ncells)), dim3(256), 0, st, s.cstart, s.ncells, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(s.ncells)), dim3(256), 0, st, s.cend, s.ncells, 0);
    hipLaunchKernelGGL(k_cell_ranges, dim3(blocks(S.N)), dim3(256), 0, st, s.keys, S.N, d * (bits - s.L), s.cstart,
                       s.cend);
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

// kNN of the centres of set C (iterated in C's search order) among set S
int run_knn(rbffd_plan* p, const Search& cs, const Search& ss, int64_t Nc, int64_t Ns, int k, int32_t* out,
            hipStream_t st) {
    const int d = p->dim;
    const int bits = d == 2 ? MORTON_BITS_2D : MORTON_BITS_3D;
    KnnArgs a{};
    a.cxyz = cs.sxyz;
    a.crow = cs.sperm;
    a.Nc = Nc;
    a.sxyz = ss.sxyz;
    a.sorig = ss.sperm;
    a.Ns = Ns;
    a.cstart = ss.cstart;
    a.cend = ss.cend;
    a.d = d;
    a.k = k;
    a.L = ss.L;
    a.bits = bits;
    for (int q = 0; q < 3; ++q) a.lo[q] = p->mlo[q];
    a.scale = std::ldexp(1.0, bits) / p->mside;
    a.side = p->mside;
    a.periodic = p->p.bc == RBFFD_BC_PERIODIC;
    for (int q = 0; q < 3; ++q) a.period[q] = p->p.hi[q] - p->p.lo[q];
    a.out = out;
    const dim3 g(blocks(Nc, 64)), b(64);
    if (k <= 32) hipLaunchKernelGGL(k_knn<32>, g, b, 0, st, a);
    else if (k <= 64) hipLaunchKernelGGL(k_knn<64>, g, b, 0, st, a);
    else hipLaunchKernelGGL(k_knn<128>, g, b, 0, st, a);
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

// Reverse Cuthill-McKee on the host from the curl stencils (original labels):
// start at the unvisited node of smallest (degree, id), breadth first,
// neighbours in increasing (degree, id), every component, then reverse.
std::vector<int32_t> rcm_host(const std::vector<int32_t>& knn, int64_t N, int width, int ncurl) {
    std::vector<std::vector<int32_t>> nb(N);
    for (int64_t i = 0; i < N; ++i)
        for (int s = 0; s < ncurl; ++s) {
            const int32_t j = knn[i * width + s];
            if (j != i) {
                nb[i].push_back(j);
                nb[j].push_back((int32_t)i);
            }
        }
    std::vector<int32_t> deg(N);
    for (int64_t i = 0; i < N; ++i) {
        std::sort(nb[i].begin(), nb[i].end());
        nb[i].erase(std::unique(nb[i].begin(), nb[i].end()), nb[i].end());
        deg[i] = (int32_t)nb[i].size();
    }
    auto less = [&](int32_t a, int32_t b) { return deg[a] < deg[b] || (deg[a] == deg[b] && a < b); };
    std::vector<int32_t> by(N);
    std::iota(by.begin(), by.end(), 0);
    std::sort(by.begin(), by.end(), less);
    std::vector<char> vis(N, 0);
    std::vector<int32_t> order;
    order.reserve(N);
    std::vector<int32_t> tmp;
    for (int32_t s0 : by) {
        if (vis[s0]) continue;
        vis[s0] = 1;
        size_t head = order.size();
        order.push_back(s0);
        while (head < order.size()) {
            const int32_t v = order[head++];
            tmp.clear();
            for (int32_t u : nb[v])
                if (!vis[u]) tmp.push_back(u);
            std::sort(tmp.begin(), tmp.end(), less);
            for (int32_t u : tmp) {
                vis[u] = 1;
                order.push_back(u);
            }
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

}  // namespace

// ---------------------------------------------------------------------------
int64_t setup_ws_bytes(const rbffd_plan* p) {
    WS w{nullptr};
    Search a{}, b{};
    const bool per = p->p.bc == RBFFD_BC_PERIODIC;
    take_search(w, a, p->E.N, p->dim, p->ns, per);
    if (!p->collocated) take_search(w, b, p->H.N, p->dim, p->ns, per);
    // kNN outputs (original labels)
    if (p->collocated) {
        w.take<int32_t>(p->E.N * p->ns);
    } else {
        w.take<int32_t>(p->H.N * p->n);
        w.take<int32_t>(p->H.N * std::max(p->nh, 1));
        w.take<int32_t>(p->E.N * p->n);
        w.take<int32_t>(p->E.N * std::max(p->nh, 1));
    }
    w.take<int32_t>(64);   // status
    if (has_wall_normals(p)) w.take<double>(p->E.N * p->dim);   // normals, original order
    int64_t need = w.off;
    if (p->collocated) {
        WS t{nullptr};
        const int64_t E = p->E.N * p->ns;
        t.take<uint64_t>(E);
        t.take<uint64_t>(E);
        t.take<int32_t>(E);
        t.take<int32_t>(E);
        t.take<char>((int64_t)key_sort_temp_bytes(E));
        t.take<char>((int64_t)scan_temp_bytes(E));
        need = std::max(need, t.off);
    }
    if (p->p.adjoint) {
        WS t{nullptr};
        const int64_t E = p->E.N * p->ns;
        t.take<uint64_t>(E);
        t.take<uint64_t>(E);
        t.take<int32_t>(p->E.N);
        t.take<int32_t>(p->E.N);
        t.take<char>((int64_t)key_sort_temp_bytes(E));
        need = std::max(need, t.off);
    }
    return align_up(need, 256) + 4096;
}

static int stage_status(rbffd_plan* p, int32_t* status, hipStream_t s) {
    int32_t h[2];
    HIPCHK(p, hipMemcpyAsync(h, status, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(p, hipStreamSynchronize(s));
    if (h[1] != 0)
        return set_err(p, RBFFD_ESINGULAR, "duplicate node positions: " + std::to_string(h[1]) +
                                               " nodes are not first in their own stencil");
    if (h[0] != INT32_MAX)
        return set_err(p, RBFFD_ESINGULAR, "singular local system at internal node " + std::to_string(h[0]));
    return RBFFD_OK;
}

// Node reordering and stencils; weights; packing -- driven by rbffd_weights.
int setup_nodes_and_stencils(rbffd_plan* p, void* wsp, hipStream_t st) {
    WS w{(char*)wsp};
    const bool per = p->p.bc == RBFFD_BC_PERIODIC;
    const int d = p->dim;
    Search se{}, sh{};
    take_search(w, se, p->E.N, d, p->ns, per);
    if (!p->collocated) take_search(w, sh, p->H.N, d, p->ns, per);
    int32_t *kE = nullptr, *kHc = nullptr, *kHh = nullptr, *kEc = nullptr, *kEh = nullptr;
    if (p->collocated) {
        kE = w.take<int32_t>(p->E.N * p->ns);
    } else {
        kHc = w.take<int32_t>(p->H.N * p->n);
        kHh = w.take<int32_t>(p->H.N * std::max(p->nh, 1));
        kEc = w.take<int32_t>(p->E.N * p->n);
        kEh = w.take<int32_t>(p->E.N * std::max(p->nh, 1));
    }
    int32_t* status = w.take<int32_t>(64);
    double* nrm_in = has_wall_normals(p) ? w.take<double>(p->E.N * d) : nullptr;   // original order
    // upload node data
    HIPCHK(p, hipMemcpyAsync(p->E.xyz_in, p->E.xyz_host.data(), p->E.N * d * 8, hipMemcpyHostToDevice, st));
    HIPCHK(p, hipMemcpyAsync(p->E.flags_in, p->E.flags_host.data(), p->E.N, hipMemcpyHostToDevice, st));
    if (nrm_in) {
        const size_t nb = (size_t)p->E.N * d * 8;
        if (p->E.nrm_host.empty()) HIPCHK(p, hipMemsetAsync(nrm_in, 0, nb, st));
        else HIPCHK(p, hipMemcpyAsync(nrm_in, p->E.nrm_host.data(), nb, hipMemcpyHostToDevice, st));
    }
    int rc = build_search(p, p->E, se, st);
    if (rc) return rc;
    if (!p->collocated) {
        HIPCHK(p, hipMemcpyAsync(p->H.xyz_in, p->H.xyz_host.data(), p->H.N * d * 8, hipMemcpyHostToDevice, st));
        HIPCHK(p, hipMemcpyAsync(p->H.flags_in, p->H.flags_host.data(), p->H.N, hipMemcpyHostToDevice, st));
        rc = build_search(p, p->H, sh, st);
        if (rc) return rc;
    }
    // stencils in original labels
    if (p->collocated) {
        rc = run_knn(p, se, se, p->E.N, p->E.N, p->ns, kE, st);
        if (rc) return rc;
    } else {
        if ((rc = run_knn(p, sh, se, p->H.N, p->E.N, p->n, kHc, st))) return rc;
        if (p->nh > 0 && (rc = run_knn(p, sh, sh, p->H.N, p->H.N, p->nh, kHh, st))) return rc;
        if ((rc = run_knn(p, se, sh, p->E.N, p->H.N, p->n, kEc, st))) return rc;
        if (p->nh > 0 && (rc = run_knn(p, se, se, p->E.N, p->E.N, p->nh, kEh, st))) return rc;
    }
    // internal order
    auto order_set = [&](NodeSet& S, Search& s) -> int {
        if (p->p.reorder == RBFFD_ORDER_MORTON) {
            HIPCHK(p, hipMemcpyAsync(S.perm, s.sperm, S.N * 4, hipMemcpyDeviceToDevice, st));
        } else if (p->p.reorder == RBFFD_ORDER_NONE || !p->collocated) {
            hipLaunchKernelGGL(k_iota, dim3(blocks(S.N)), dim3(256), 0, st, S.perm, S.N);
        } else {
            std::vector<int32_t> kh(S.N * p->ns);
            HIPCHK(p, hipMemcpyAsync(kh.data(), kE, S.N * p->ns * 4, hipMemcpyDeviceToHost, st));
            HIPCHK(p, hipStreamSynchronize(st));
            std::vector<int32_t> order = rcm_host(kh, S.N, p->ns, p->n);
            HIPCHK(p, hipMemcpyAsync(S.perm, order.data(), S.N * 4, hipMemcpyHostToDevice, st));
            HIPCHK(p, hipStreamSynchronize(st));
        }
        hipLaunchKernelGGL(k_inverse, dim3(blocks(S.N)), dim3(256), 0, st, S.perm, S.N, S.inv);
        hipLaunchKernelGGL(k_internal_nodes, dim3(blocks(S.N)), dim3(256), 0, st, S.xyz_in, S.flags_in, S.perm, S.N, d,
                           S.xyz, S.emask, (int)per, (int)(p->p.pol == RBFFD_POL_TE),
                           &S == &p->E ? nrm_in : nullptr, S.nrm);
        return RBFFD_OK;
    };
    if (p->p.reorder == RBFFD_ORDER_RCM && !p->collocated)
        return set_err(p, RBFFD_ENOTSUP, "RCM ordering is implemented for collocated plans");
    if ((rc = order_set(p->E, se))) return rc;
    if (!p->collocated && (rc = order_set(p->H, sh))) return rc;
    if (p->collocated) {
        hipLaunchKernelGGL(k_relabel, dim3(blocks(p->E.N)), dim3(256), 0, st, kE, p->ns, p->E.perm, p->E.inv, p->E.N,
                           p->opH.st_union, p->ns);
    } else {
        hipLaunchKernelGGL(k_relabel, dim3(blocks(p->H.N)), dim3(256), 0, st, kHc, p->n, p->H.perm, p->E.inv, p->H.N,
                           p->opH.st_curl, p->n);
        hipLaunchKernelGGL(k_relabel, dim3(blocks(p->E.N)), dim3(256), 0, st, kEc, p->n, p->E.perm, p->H.inv, p->E.N,
                           p->opE.st_curl, p->n);
        if (p->nh > 0) {
            hipLaunchKernelGGL(k_relabel, dim3(blocks(p->H.N)), dim3(256), 0, st, kHh, p->nh, p->H.perm, p->H.inv,
                               p->H.N, p->opH.st_hv, p->nh);
            hipLaunchKernelGGL(k_relabel, dim3(blocks(p->E.N)), dim3(256), 0, st, kEh, p->nh, p->E.perm, p->E.inv,
                               p->E.N, p->opE.st_hv, p->nh);
        }
    }
    (void)status;
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

static int launch_weights(rbffd_plan* p, const OpBlock& o, const NodeSet& T, const NodeSet& S, bool curl,
                          int32_t* status, hipStream_t st) {
    const int d = p->dim;
    WArgs a{};
    a.txyz = T.xyz;
    a.sxyz = S.xyz;
    a.d = d;
    a.periodic = p->p.bc == RBFFD_BC_PERIODIC;
    for (int k = 0; k < 3; ++k) a.period[k] = p->p.hi[k] - p->p.lo[k];
    a.Nt = o.Nt;
    a.status = status;
    if (curl) {
        a.st = o.cross ? o.st_curl : o.st_union;
        a.st_stride = o.cross ? o.n : o.ns;
        a.n = o.n;
        a.M = p->M;
        a.kind = (p->p.mode == RBFFD_MODE_VFD) ? W_VFD : W_FD;
        a.phs_k = p->p.phs_k;
        a.nrhs = d;
        a.upow = 1;
        a.vdelta = p->p.vfd_sigma * p->p.h;
        for (int q = 0; q < 3; ++q)
            for (int k = 0; k < 3; ++k) a.fu[q][k] = (q == k) ? 1.0 : 0.0;
        if (p->p.frame_angle != 0.0) {
            const double cs = std::cos(p->p.frame_angle), sn = std::sin(p->p.frame_angle);
            a.fu[0][0] = cs;
            a.fu[0][1] = sn;
            a.fu[1][0] = -sn;
            a.fu[1][1] = cs;
        }
        for (int q = 0; q < p->M; ++q)
            for (int k = 0; k < 3; ++k) a.ex[q][k] = (int8_t)p->ex_m[q][k];
        a.out = o.wc;
        a.check_self = !o.cross;
    } else {
        const int al = p->p.hv_alpha;
        a.st = o.cross ? o.st_hv : o.st_union;
        a.st_stride = o.cross ? o.nh : o.ns;
        a.n = o.nh;
        a.M = p->Mh;
        a.kind = W_HV;
        a.phs_k = 2 * al + 1;
        a.nrhs = 1;
        a.upow = 2 * al;
        // Delta^alpha r^k = C r^(k - 2 alpha): radial Laplacian k (k + d - 2) r^(k-2), iterated
        double C = 1.0;
        for (int t = 0, kk = a.phs_k; t < al; ++t, kk -= 2) C *= (double)kk * (kk + d - 2);
        a.hv_C = C;
        for (int q = 0; q < p->Mh; ++q) {
            for (int k = 0; k < 3; ++k) a.ex[q][k] = (int8_t)p->ex_h[q][k];
            // Delta^alpha x^a y^b z^c at 0: nonzero only for a = 2i, b = 2j, c = 2l with i + j + l = alpha;
            // value alpha! / (i! j! l!) * a! b! c!
            const int* e = p->ex_h[q];
            double v = 0.0;
            if (e[0] + e[1] + e[2] == 2 * al && e[0] % 2 == 0 && e[1] % 2 == 0 && e[2] % 2 == 0) {
                auto fact = [](int x) { double f = 1; for (int i = 2; i <= x; ++i) f *= i; return f; };
                v = fact(al) / (fact(e[0] / 2) * fact(e[1] / 2) * fact(e[2] / 2)) * fact(e[0]) * fact(e[1]) * fact(e[2]);
            }
            a.hv_poly[q] = v;
        }
        a.out = o.wh;
        a.check_self = 1;
    }
    const int R = a.n + a.M;
    constexpr int64_t chunk = (int64_t)1 << 21;   // a dispatch counts work-items in 32 bits
    if (R + a.nrhs <= WREG_MAX) {
        // the system fits the register-resident solver (every configured
        // workload), with the smallest register block that holds it
        const int blk = (R + a.nrhs + WREG_T - 1) / WREG_T;
        for (int64_t c0 = 0; c0 < o.Nt; c0 += chunk) {
            a.c0 = c0;
            const int64_t nb = std::min<int64_t>(chunk, o.Nt - c0);
            if (blk <= 3) hipLaunchKernelGGL(k_wreg<3>, dim3((unsigned)nb), dim3(256), 0, st, a);
            else if (blk <= 4) hipLaunchKernelGGL(k_wreg<4>, dim3((unsigned)nb), dim3(256), 0, st, a);
            else if (blk <= 6) hipLaunchKernelGGL(k_wreg<6>, dim3((unsigned)nb), dim3(256), 0, st, a);
            else hipLaunchKernelGGL(k_wreg<7>, dim3((unsigned)nb), dim3(256), 0, st, a);
            HIPCHK(p, hipGetLastError());
        }
        return RBFFD_OK;
    }
    const size_t lds = (size_t)(R * (R + a.nrhs) + a.n * 3 + R) * 8;
    int dev = 0, max_lds = 65536;
    HIPCHK(p, hipGetDevice(&dev));
    HIPCHK(p, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (lds + 64 > (size_t)max_lds)
        return set_err(p, RBFFD_ESIZE, "local system of " + std::to_string(R) + " unknowns needs " +
                                           std::to_string(lds) + " B of LDS; the device allows " +
                                           std::to_string(max_lds));
    // larger systems: 16 wavefronts per system with the matrix in LDS; the
    // elimination steps are chains of LDS round trips, so more wavefronts hide
    // more of their latency (at most 2^21 systems per launch, as above)
    for (int64_t c0 = 0; c0 < o.Nt; c0 += chunk) {
        a.c0 = c0;
        const int64_t nb = std::min<int64_t>(chunk, o.Nt - c0);
        hipLaunchKernelGGL(k_weights, dim3((unsigned)nb), dim3(1024), lds, st, a);
        HIPCHK(p, hipGetLastError());
    }
    return RBFFD_OK;
}

int setup_weights(rbffd_plan* p, void* wsp, hipStream_t st) {
    WS w{(char*)wsp};
    int32_t* status = w.take<int32_t>(64);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, status, 64, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, st, status, 1, INT32_MAX);
    int rc;
    if (p->collocated) {
        if ((rc = launch_weights(p, p->opH, p->E, p->E, true, status, st))) return rc;
        if (p->nh > 0 && (rc = launch_weights(p, p->opH, p->E, p->E, false, status, st))) return rc;
    } else {
        if ((rc = launch_weights(p, p->opH, p->H, p->E, true, status, st))) return rc;
        if (p->nh > 0 && (rc = launch_weights(p, p->opH, p->H, p->H, false, status, st))) return rc;
        if ((rc = launch_weights(p, p->opE, p->E, p->H, true, status, st))) return rc;
        if (p->nh > 0 && (rc = launch_weights(p, p->opE, p->E, p->E, false, status, st))) return rc;
    }
    return stage_status(p, status, st);
}

static int pack_block(rbffd_plan* p, const OpBlock& o, hipStream_t st) {
    const int d = p->dim;
    const int64_t G = o.tiles * RBFFD_TILE;
    const bool f64 = p->p.wdtype == RBFFD_F64;
    if (!o.cross) {
        if (p->p.wdtype == RBFFD_W22)
            hipLaunchKernelGGL(k_pack_union<w22>, dim3(blocks(G)), dim3(256), 0, st, o.st_union, o.wc, o.wh, o.Nt,
                               o.ns, o.n, o.nh, d, o.C4, o.V4, o.S4, o.tiles, (int4*)o.pidx, (w22*)o.pwc,
                               (w22*)o.pwh);
        else if (f64)
            hipLaunchKernelGGL(k_pack_union<double>, dim3(blocks(G)), dim3(256), 0, st, o.st_union, o.wc, o.wh, o.Nt,
                               o.ns, o.n, o.nh, d, o.C4, o.V4, o.S4, o.tiles, (int4*)o.pidx, (double*)o.pwc,
                               (double*)o.pwh);
        else
            hipLaunchKernelGGL(k_pack_union<float>, dim3(blocks(G)), dim3(256), 0, st, o.st_union, o.wc, o.wh, o.Nt,
                               o.ns, o.n, o.nh, d, o.C4, o.V4, o.S4, o.tiles, (int4*)o.pidx, (float*)o.pwc,
                               (float*)o.pwh);
        if (p->K > 1)
            hipLaunchKernelGGL(k_pack_batched, dim3(blocks(o.Nt)), dim3(256), 0, st, o.st_union, o.wc, o.wh, o.Nt, o.ns,
                               o.n, o.nh, d, o.C4, o.V4, o.S4, o.bidx, o.bwc, o.bwh, o.bw0);
    } else {
        if (f64)
            hipLaunchKernelGGL(k_pack_cross<double>, dim3(blocks(G)), dim3(256), 0, st, o.st_curl, o.st_hv, o.wc, o.wh,
                               o.Nt, o.n, o.nh, d, o.C4, o.V4, o.tiles, (int4*)o.pidx, (int4*)o.pidx_h, o.pref,
                               (double*)o.pwc, (double*)o.pwh);
        else
            hipLaunchKernelGGL(k_pack_cross<float>, dim3(blocks(G)), dim3(256), 0, st, o.st_curl, o.st_hv, o.wc, o.wh,
                               o.Nt, o.n, o.nh, d, o.C4, o.V4, o.tiles, (int4*)o.pidx, (int4*)o.pidx_h, o.pref,
                               (float*)o.pwc, (float*)o.pwh);
    }
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}

int pack_all(rbffd_plan* p, void*, hipStream_t st) {
    int rc = pack_block(p, p->opH, st);
    if (rc) return rc;
    if (!p->collocated) rc = pack_block(p, p->opE, st);
    return rc;
}

int build_transpose(rbffd_plan* p, void* wsp, hipStream_t st) {
    OpBlock& o = p->opH;
    const int64_t N = o.Nt, ns = o.ns, E = N * ns;
    WS w{(char*)wsp};
    uint64_t* kin = w.take<uint64_t>(E);
    uint64_t* kout = w.take<uint64_t>(E);
    int32_t* rstart = w.take<int32_t>(N);
    int32_t* rend = w.take<int32_t>(N);
    size_t tb = key_sort_temp_bytes(E);
    void* temp = w.take<char>((int64_t)tb);
    hipLaunchKernelGGL(k_tkeys, dim3(blocks(E)), dim3(256), 0, st, o.st_union, N, (int)ns, kin);
    int end_bit = 1;
    while (end_bit < 64 && ((uint64_t)1 << end_bit) <= (uint64_t)(N * E)) ++end_bit;
    HIPCHK(p, rocprim::radix_sort_keys(temp, tb, kin, kout, (int)E, 0, (unsigned)std::min(end_bit + 1, 64), st));
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(N)), dim3(256), 0, st, rstart, N, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(N)), dim3(256), 0, st, rend, N, 0);
    hipLaunchKernelGGL(k_tdeg, dim3(blocks(E)), dim3(256), 0, st, kout, E, N * ns, rstart, rend);
    hipLaunchKernelGGL(k_twidth, dim3(blocks(o.tiles)), dim3(256), 0, st, rstart, rend, N, o.tiles, o.t_width);
    std::vector<int32_t> width(o.tiles);
    HIPCHK(p, hipMemcpyAsync(width.data(), o.t_width, o.tiles * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    std::vector<int64_t> off(o.tiles + 1, 0);
    for (int64_t t = 0; t < o.tiles; ++t) off[t + 1] = off[t] + (int64_t)width[t] * RBFFD_TILE;
    if (off[o.tiles] > o.t_cap) return set_err(p, RBFFD_ESIZE, "transposed operator exceeds its capacity");
    HIPCHK(p, hipMemcpyAsync(o.t_off, off.data(), (o.tiles + 1) * 8, hipMemcpyHostToDevice, st));
    const int64_t G = o.tiles * RBFFD_TILE;
    hipLaunchKernelGGL(k_tfill, dim3(blocks(G)), dim3(256), 0, st, kout, rstart, rend, o.t_off, o.t_width, N, (int)ns,
                       o.tiles, o.t_src, o.t_slot);
    p->t_entries = off[o.tiles];
    int rc = refill_transpose(p, st);
    if (rc) return rc;
    HIPCHK(p, hipGetLastError());
    HIPCHK(p, hipStreamSynchronize(st));
    p->opE = p->opH;
    return RBFFD_OK;
}

int build_halos(rbffd_plan* p, void* wsp, hipStream_t st) {
    OpBlock& o = p->opH;
    o.hmax = 0;
    if (!o.lidx) return RBFFD_OK;
    const int64_t N = o.Nt, ns = o.ns, E = N * ns;
    if (E > INT32_MAX) return RBFFD_OK;   // too many entries for the 32-bit scan: no staging
    WS w{(char*)wsp};
    uint64_t* kin = w.take<uint64_t>(E);
    uint64_t* kout = w.take<uint64_t>(E);
    int32_t* flag = w.take<int32_t>(E);
    int32_t* pos = w.take<int32_t>(E);
    size_t tb = key_sort_temp_bytes(E), sb = scan_temp_bytes(E);
    void* temp = w.take<char>((int64_t)tb);
    void* stemp = w.take<char>((int64_t)sb);
    const bool batch = p->K > 1;
    const int tsz = o.wgt;
    hipLaunchKernelGGL(k_hkeys, dim3(blocks(E)), dim3(256), 0, st, o.st_union, N, (int)ns, tsz, kin);
    int end_bit = 32;
    while (end_bit < 64 && ((uint64_t)1 << (end_bit - 32)) <= (uint64_t)o.nwg) ++end_bit;
    HIPCHK(p, rocprim::radix_sort_keys(temp, tb, kin, kout, (int)E, 0, (unsigned)end_bit, st));
    hipLaunchKernelGGL(k_hflags, dim3(blocks(E)), dim3(256), 0, st, kout, E, flag);
    HIPCHK(p, rocprim::exclusive_scan(stemp, sb, flag, pos, (int32_t)0, (size_t)E, rocprim::plus<int32_t>(), st));
    hipLaunchKernelGGL(k_hcompact, dim3(blocks(E)), dim3(256), 0, st, kout, flag, pos, E, o.hpool, o.hoff, o.nwg);
    hipLaunchKernelGGL(k_hlocal, dim3(blocks(o.tiles * RBFFD_TILE)), dim3(256), 0, st, o.st_union, N, (int)ns,
                       o.hpool, o.hoff, o.Q8, o.tiles, tsz, o.lidx, o.lself);
    HIPCHK(p, hipGetLastError());
    std::vector<int32_t> off(o.nwg + 1);
    HIPCHK(p, hipMemcpyAsync(off.data(), o.hoff, (o.nwg + 1) * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    int32_t mx = 0;
    for (int64_t t = 0; t < o.nwg; ++t) mx = std::max(mx, off[t + 1] - off[t]);
    // staging only when a workgroup's list fits the LDS budget and 16-bit positions
    o.stage = 0;
    o.hmax = 0;
    if (mx < 65536) {
        const int64_t fb = field_elem_bytes(p->p.fdtype) == 8 ? 8 : 4;
        if (batch) {
            // an 8-field slice per component
            if ((int64_t)mx * (p->fe_comp + p->fh_comp) * 8 * 4 <= RBFFD_LDS_BUDGET_BATCH) o.hmax = mx;
        } else if (p->dim == 2) {
            // E values (rounded up to 4 entries) and (Hx, Hy) pairs, as the 2D kernels lay them out
            if ((((int64_t)mx + 3) / 4 * 4 + 2 * (int64_t)mx) * fb <= RBFFD_LDS_BUDGET) o.stage = 1;
        } else {
            // packed 3-vectors: both fields together, else one at a time
            if (6 * (int64_t)mx * fb <= RBFFD_LDS_BUDGET_3D) o.stage = 1;
            else if (3 * (int64_t)mx * fb <= RBFFD_LDS_BUDGET) o.stage = 2;
        }
        if (o.stage) o.hmax = mx;
    }
    p->opE = p->opH;
    return RBFFD_OK;
}

int refill_transpose(rbffd_plan* p, hipStream_t st) {
    OpBlock& o = p->opH;
    const int64_t E = p->t_entries;
    if (E <= 0) return RBFFD_OK;
    if (p->p.wdtype == RBFFD_F64)
        hipLaunchKernelGGL(k_tweights<double>, dim3(blocks(E)), dim3(256), 0, st, o.t_src, o.t_slot, E, o.wc, o.wh,
                           o.n, o.nh, o.t_cap, (double*)o.t_w);
    else
        hipLaunchKernelGGL(k_tweights<float>, dim3(blocks(E)), dim3(256), 0, st, o.t_src, o.t_slot, E, o.wc, o.wh,
                           o.n, o.nh, o.t_cap, (float*)o.t_w);
    HIPCHK(p, hipGetLastError());
    p->opE = p->opH;
    return RBFFD_OK;
}

// ---------------------------------------------------------------------------
// Public set-up entry point and the permutation helper
// ---------------------------------------------------------------------------
extern "C" int rbffd_weights(rbffd_plan* p, void* arena, void* ws, void* stream) {
    if (!p || !arena || !ws) return RBFFD_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    p->arena = (char*)arena;
    p->ready = false;
    int64_t wsb = 0, aws = 0;
    layout_arena(p, p->arena, &wsb, &aws);
    int rc = setup_nodes_and_stencils(p, ws, st);
    if (rc) return rc;
    if ((rc = setup_weights(p, ws, st))) return rc;
    if ((rc = pack_all(p, ws, st))) return rc;
    if (p->collocated && (rc = build_halos(p, ws, st))) return rc;
    if (p->p.adjoint && (rc = build_transpose(p, ws, st))) return rc;
    if (p->K > 1 && (rc = fill_field_gamma(p, nullptr, st))) return rc;
    HIPCHK(p, hipStreamSynchronize(st));
    p->ready = true;
    return RBFFD_OK;
}

__global__ void k_permute(const char* in, char* out, const int32_t* perm, int64_t N, int64_t eb, int to_internal) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t words = eb / 2;
    if (g >= N * words) return;
    const int64_t p = g / words, w = g % words;
    const int64_t o = perm[p];
    const uint16_t* src = (const uint16_t*)in;
    uint16_t* dst = (uint16_t*)out;
    if (to_internal) dst[p * words + w] = src[o * words + w];
    else dst[o * words + w] = src[p * words + w];
}

extern "C" int rbffd_permute(const rbffd_plan* p, int32_t set, int32_t to_internal, int64_t eb, const void* in,
                             void* out, void* stream) {
    if (!p || !in || !out || eb <= 0 || (eb % 2)) return RBFFD_EINVAL;
    if (!p->ready) return set_err(p, RBFFD_ESTATE, "rbffd_weights has not run");
    if (in == out) return set_err(p, RBFFD_EINVAL, "permute cannot work in place");
    const NodeSet& S = (set == 1 && !p->collocated) ? p->H : p->E;
    const int64_t n = S.N * (eb / 2);
    hipLaunchKernelGGL(k_permute, dim3(blocks(n)), dim3(256), 0, (hipStream_t)stream, (const char*)in, (char*)out,
                       S.perm, S.N, eb, to_internal);
    HIPCHK(p, hipGetLastError());
    return RBFFD_OK;
}
