/*
 * rbffd.h -- C ABI of the MI355X (gfx950) meshless FDTD library.
 *
 * The library advances Maxwell's curl equations on scattered nodes with the
 * stabilised interleaved leapfrog of Kolar-Pozun & Kosec, "An RBF-based
 * method for computational electromagnetics with reduced numerical
 * dispersion" (arXiv 2508.18205), Section 5, eq. 19, using precomputed local
 * RBF differentiation weights (Section 4, eq. 9-15) for the curl and the
 * hyperviscosity operator (Section 5.1).
 *
 * Conventions shared by every call
 *  - Return value: RBFFD_OK (0) or a negative RBFFD_E* code; the plan keeps a
 *    human-readable message (rbffd_last_error).  Nothing throws across the ABI.
 *  - Memory: the CALLER owns all device memory.  rbffd_plan_sizes reports how
 *    many bytes each buffer needs; the library never allocates device memory.
 *    Host pointers are marked _host, everything else is device memory.
 *  - Streams: every device call is asynchronous on the hipStream_t passed as
 *    `void* stream` (NULL = the null stream).  Calls that return host data
 *    synchronise that stream before returning.
 *  - Node order: device state arrays are in the plan's INTERNAL order (the
 *    node reordering chosen in rbffd_params.reorder).  rbffd_get_perm and
 *    rbffd_permute convert to and from the caller's (original) order.
 *  - Threading: a plan may be used by one host thread at a time.
 */
#ifndef RBFFD_H
#define RBFFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define RBFFD_OK          0
#define RBFFD_EINVAL     -1   /* bad argument or parameter combination       */
#define RBFFD_ESIZE      -2   /* a size or count exceeds a supported maximum */
#define RBFFD_ESINGULAR  -3   /* a local weight system is singular           */
#define RBFFD_EHIP       -4   /* a HIP runtime call failed                   */
#define RBFFD_EUNSTABLE  -5   /* NaN/Inf or energy above the run threshold   */
#define RBFFD_ESTATE     -6   /* call out of order (e.g. step before weights)*/
#define RBFFD_ENOTSUP    -7   /* feature not supported for this plan         */

/* ---- enumerations ------------------------------------------------------ */
#define RBFFD_MODE_FD     0   /* RBF-FD curl weights, eq. 13 (collocated)      */
#define RBFFD_MODE_VFD    1   /* RBF-VFD central virtual difference, eq. 15    */
#define RBFFD_MODE_STAG2  2   /* E and H on two node sets, RBF-FD (not the
                                 paper's choice; cross-set curl stencils)     */
#define RBFFD_BC_PEC      0   /* perfectly conducting walls on flagged nodes  */
#define RBFFD_BC_PERIODIC 1   /* periodic box [lo, hi) (minimum image)        */
/* 2D polarisation.  TEz (Ex, Ey, Hz) uses the same leapfrog and
 * hyperviscosity as TMz with the fields' roles exchanged:
 *   Hz <- Hz - a (D^dx Ey - D^dy Ex - gamma D^hv Hz)
 *   Ex <- Ex + kappa (D^dy Hz_new + gamma D^hv Ex)
 *   Ey <- Ey + kappa (-D^dx Hz_new + gamma D^hv Ey)
 * (Hz at half steps); a wall flagged as normal to x zeroes Ey, one normal to
 * y zeroes Ex (axis-aligned walls; curved walls take per-node normals, see
 * rbffd_set_wall_normals).  Sources, receivers, the K-field batch,
 * the adjoint and the two-set variant are TMz only. */
#define RBFFD_POL_TM 0
#define RBFFD_POL_TE 1
#define RBFFD_ORDER_NONE   0
#define RBFFD_ORDER_MORTON 1
#define RBFFD_ORDER_RCM    2
#define RBFFD_F64  0
#define RBFFD_F32  1
#define RBFFD_BF16 2          /* field storage only; arithmetic in FP32       */
#define RBFFD_W22  3          /* weight storage only (wdtype): compressed FP32
                                 weights, four 22-bit mantissas and one shared
                                 exponent per 4-slot chunk (12 bytes instead of
                                 16); FP32 fields and arithmetic; 2D collocated
                                 single-field plans without the adjoint      */

/* Which operator rbffd_get_weights / rbffd_set_weights address.  For the
 * two-set variant the *_H operators are the ones applied in the H update
 * (centres on the H set) and *_E in the E update. */
#define RBFFD_OP_CURL_H 0     /* [N_target][dim][n]  first-derivative weights */
#define RBFFD_OP_HV_H   1     /* [N_target][n_hv]    Delta^alpha weights      */
#define RBFFD_OP_CURL_E 2
#define RBFFD_OP_HV_E   3

/* Which stencil rbffd_get_stencils returns (internal labels). */
#define RBFFD_ST_UNION   0    /* collocated: [N][n_stencil], n_stencil = max(n, n_hv) */
#define RBFFD_ST_CURL_H  1    /* two-set: [N_H][n] indices into the E set     */
#define RBFFD_ST_HV_H    2    /* two-set: [N_H][n_hv] indices into the H set  */
#define RBFFD_ST_CURL_E  3    /* two-set: [N_E][n] indices into the H set     */
#define RBFFD_ST_HV_E    4    /* two-set: [N_E][n_hv] indices into the E set  */

/* ---- parameters -------------------------------------------------------- */
/* Every parameter of the method (Section 4.3, Section 5, Section 5.1). */
typedef struct rbffd_params {
    int32_t dim;        /* 2 = TMz (eq. 3) or TEz (see pol), 3 = full curl eqs.  */
    int32_t mode;       /* RBFFD_MODE_*                                           */
    int32_t n;          /* curl stencil size (n nearest nodes, eq. 11)            */
    int32_t m;          /* curl monomial degree (eq. 8)                           */
    int32_t phs_k;      /* curl PHS exponent, phi(r) = r^phs_k (odd, >= 3)         */
    int32_t hv_alpha;   /* hyperviscosity power alpha (0 = none)                  */
    int32_t n_hv;       /* HV stencil size; 0 = 2 * C(2 alpha + dim, dim) + 1      */
    int32_t bc;         /* RBFFD_BC_*                                             */
    int32_t reorder;    /* RBFFD_ORDER_*                                          */
    int32_t wdtype;     /* stored weight precision for the step: F64, F32 or W22   */
    int32_t fdtype;     /* field storage: F64, F32 or BF16 (BF16 needs F32 weights)*/
    int32_t K;          /* independent fields per batch (1 = single field; 2D)    */
    int32_t adjoint;    /* nonzero: also build transposed operators (2D, K = 1)   */
    int32_t pol;        /* 2D polarisation: RBFFD_POL_TM (Ez, Hx, Hy) or
                           RBFFD_POL_TE (Ex, Ey, Hz; collocated, K = 1)           */
    double vfd_sigma;   /* RBF-VFD virtual spacing delta = vfd_sigma * h          */
    double hv_c;        /* c of gamma = c (-1)^(alpha-1) h^(2 alpha), units 1/time */
    double h;           /* nominal node spacing of the E set                      */
    double h_h;         /* nominal spacing of the H set (two-set only; 0 = h)     */
    double dt;          /* time step; 0 = h / (10 sqrt(2) c0)                     */
    double eps0, mu0;   /* vacuum constants (c0 = 1/sqrt(eps0 mu0))               */
    double lo[3], hi[3];/* bounding box; the period for RBFFD_BC_PERIODIC         */
    double frame_angle; /* 2D only (0 in 3D): angle theta of the frame the curl is
                           discretised in (the angle study of Section 6, eq. 27).
                           The two derivative operators act along
                           u1 = (cos theta, sin theta), u2 = (-sin theta, cos
                           theta), and field vectors are stored in components
                           along u1, u2; RBF-VFD puts its virtual points at
                           +-delta u.  0 = the x and y axes.                     */
} rbffd_params;

/* Sizes of every caller-owned buffer, in bytes, plus derived constants. */
typedef struct rbffd_sizes {
    int64_t N;               /* nodes of the E set (= all nodes when collocated) */
    int64_t N_h;             /* nodes of the H set (= N when collocated)         */
    int32_t n_stencil;       /* collocated union stencil width max(n, n_hv)      */
    int32_t n_hv;            /* effective HV stencil size                        */
    int32_t fe, fh;          /* values per node in E and H buffers (2D TMz: 1, 2;
                                2D TEz: 2, 1; 3D: 4, 4 -- x, y, z and one unused
                                pad value)                                       */
    int32_t field_elem;      /* bytes per stored field value (8, 4 or 2)         */
    int32_t K;
    int64_t arena_bytes;     /* persistent device arena (weights, stencils, ...) */
    int64_t workspace_bytes; /* scratch needed by rbffd_weights and rbffd_run    */
    int64_t e_bytes;         /* one E buffer: N * fe * K * field_elem            */
    int64_t h_bytes;         /* one H buffer: N_h * fh * K * field_elem          */
    int64_t adjoint_ws_bytes;/* scratch of rbffd_adjoint excluding its segment   */
    double dt;               /* effective time step                              */
    double gamma;            /* effective hyperviscosity strength                */
} rbffd_sizes;

typedef struct rbffd_plan rbffd_plan;

/* Field state.  E[cur], H[cur] hold (E^n, H^n) with H^n = H(t_{n - 1/2});
 * the other buffer of each pair is overwritten by the next step, after which
 * cur flips.  eps_r: NULL for eps_r = 1 everywhere, else [N] per-node relative
 * permittivity in internal order, double for F64 fields and float otherwise. */
typedef struct rbffd_fields {
    void* E[2];
    void* H[2];
    int32_t cur;
    int32_t reserved;
    const void* eps_r;
} rbffd_fields;

/* Forward run (rbffd_run).  All arrays are device memory.
 *  - energy_out [floor((T-1)/energy_every) + 1] double: U^n of eq. 20 for
 *    n = 0, energy_every, ... (computed inside step n from E^n and the
 *    average of H^n and H^{n+1}); NULL or energy_every = 0 disables.
 *    K-field batch: energy_out [samples][K], one U^n per field.
 *  - soft sources: after the E bracket of step n, E (Ez in 2D) at node
 *    src_node[s] gains src_amp[s] * src_wave[n * n_src + s]; not scaled by
 *    eps_r; PEC nodes stay zero.  (2D, K = 1.)
 *  - receivers: traces[n * n_rcv + r] = E^{n+1} at rcv_node[r] (Ez in 2D).
 *  - checkpoints: if ckpt != NULL the state (E^n, H^n) is copied to slot
 *    n / ckpt_every for every n multiple of ckpt_every, n < T; one slot is
 *    e_bytes + h_bytes long (E first).
 *  - use_graph: capture the step loop in a HIP graph and replay it.
 *  - unstable_threshold: > 0 makes the run fail with RBFFD_EUNSTABLE if an
 *    energy sample is NaN or exceeds threshold * energy_out[0].
 * The plan's precision templates apply; src_amp, src_wave are double for F64
 * fields and float otherwise; traces have the same type. */
typedef struct rbffd_run_args {
    int32_t T;
    int32_t energy_every;
    double* energy_out;
    int32_t n_src;
    int32_t n_rcv;
    const int32_t* src_node;
    const void* src_amp;
    const void* src_wave;
    const int32_t* rcv_node;
    void* traces;
    void* ckpt;
    int32_t ckpt_every;
    int32_t use_graph;
    double unstable_threshold;
    int32_t step0;           /* global index of the first step (source time)    */
    int32_t reserved;
} rbffd_run_args;

/* Discrete adjoint of a forward run (2D TMz, K = 1, collocated).
 * ckpt holds the checkpoints written by a forward run with the same T, ckpt_every
 * (slot 0 = the initial state).  grad_traces [T][n_rcv] = dJ/dtraces (same type
 * as the fields).  Outputs (device double, overwritten): grad_eps [N] =
 * dJ/deps_r (internal order), grad_amp [n_src] = dJ/dsrc_amp.  seg_buf must
 * hold (ckpt_every + 1) E buffers; workspace must hold adjoint_ws_bytes. */
typedef struct rbffd_adjoint_args {
    int32_t T;
    int32_t ckpt_every;
    const void* ckpt;
    int32_t n_src;
    int32_t n_rcv;
    const int32_t* src_node;
    const void* src_amp;
    const void* src_wave;
    const int32_t* rcv_node;
    const void* grad_traces;
    double* grad_eps;
    double* grad_amp;
    void* seg_buf;
    void* workspace;
} rbffd_adjoint_args;

/* ---- plan ---------------------------------------------------------------
 * Host-only: validates the parameters (n > M_m, n_hv > M_{2 alpha}, stencils
 * no larger than the node set, supported sizes) and copies the node data.
 * xyz_host [N][dim] doubles, flags_host [N] bytes (bit 2k / 2k+1 = node on
 * the low / high wall normal to axis k; ignored for periodic boxes).  For
 * RBFFD_MODE_STAG2 pass the H set in N_h / xyzH_host / flagsH_host, else 0
 * and NULL.  Periodic boxes: every node of both sets must lie in [lo, hi)
 * (RBFFD_EINVAL otherwise).  On success *out owns a new plan (free with
 * rbffd_plan_destroy). */
int rbffd_plan_create(const rbffd_params* p, int64_t N, const double* xyz_host,
                      const uint8_t* flags_host, int64_t N_h, const double* xyzH_host,
                      const uint8_t* flagsH_host, rbffd_plan** out);
int rbffd_plan_sizes(const rbffd_plan* plan, rbffd_sizes* out);

/* Curved PEC walls where E is a vector: the TEz polarisation and 3D.
 * normals_host [N][dim] doubles in the caller's node order: a unit outward
 * (or inward) normal on each node of a curved wall, zero elsewhere.  After
 * every E update a node with a normal keeps only the normal component of E,
 * E <- (E . n) n, so the tangential E vanishes on the wall (nodes without one
 * follow the axis rule of their flags); a 3D soft source on such a node adds
 * its projection.  (TMz needs none: Ez is tangential to every in-plane wall.)
 * Host-only; call between rbffd_plan_create and rbffd_weights (RBFFD_ESTATE
 * afterwards); NULL clears.  RBFFD_ENOTSUP for plans other than collocated
 * TEz or 3D with PEC walls; RBFFD_EINVAL for a normal that is not a unit
 * vector (|n|^2 - 1 beyond 1e-9) or sits on a node without a wall flag.  The
 * plan copies the data. */
int rbffd_set_wall_normals(rbffd_plan* plan, const double* normals_host);
void rbffd_plan_destroy(rbffd_plan* plan);
const char* rbffd_strerror(int code);
const char* rbffd_last_error(const rbffd_plan* plan);

/* ---- set-up on the GPU (computed once, reused every step: Section 5) -----
 * arena: arena_bytes of device memory kept by the plan until destroyed or
 * re-set; workspace: workspace_bytes of scratch (free to reuse afterwards).
 * Runs node reordering, exact kNN stencils, the FP64 local weight systems
 * (eq. 9 with eq. 13 / eq. 15 right-hand sides, HV by RBF-FD of Delta^alpha
 * with phi = r^(2 alpha + 1), m = 2 alpha) and packs them for the step.
 * RBFFD_ESINGULAR: a local system had a zero pivot (node named in the message). */
int rbffd_weights(rbffd_plan* plan, void* arena, void* workspace, void* stream);

/* ---- parity / inspection I/O (host buffers; synchronise the stream) ------ */
/* perm_host[p] = original index of internal node p (set 0 = E, 1 = H). */
int rbffd_get_perm(const rbffd_plan* plan, int32_t set, int32_t* perm_host, void* stream);
/* which = RBFFD_ST_*: stencil rows of internal node p, nearest first, ties by
 * original index, as internal labels of the source set. */
int rbffd_get_stencils(const rbffd_plan* plan, int32_t which, int32_t* out_host, void* stream);
/* Unfolded FP64 weights in internal order (layout of RBFFD_OP_*). */
int rbffd_get_weights(const rbffd_plan* plan, int32_t op, double* out_host, void* stream);
/* Replace the FP64 weights of one operator (same layout) and re-pack them;
 * lets the step be checked with weights computed elsewhere. */
int rbffd_set_weights(rbffd_plan* plan, int32_t op, const double* in_host, void* stream);

/* Gather / scatter a per-node array between original and internal order.
 * to_internal = 1: out[p] = in[perm[p]]; 0: out[perm[p]] = in[p].
 * Each node owns elem_bytes contiguous bytes (a multiple of 2). */
int rbffd_permute(const rbffd_plan* plan, int32_t set, int32_t to_internal, int64_t elem_bytes,
                  const void* in, void* out, void* stream);

/* ---- the hot path ---------------------------------------------------------
 * rbffd_step: nsteps full leapfrog steps (H update, then E update; eq. 19)
 * with no sources or diagnostics.  Flips f->cur once per step. */
int rbffd_step(const rbffd_plan* plan, rbffd_fields* f, int32_t nsteps, void* stream);
/* rbffd_half: one half update without flipping f->cur: which = 0 writes
 * H[1-cur] from (E[cur], H[cur]) (the H lines of eq. 19); which = 1 writes
 * E[1-cur] from (E[cur], H[1-cur]) (the E line).  rbffd_step is the pair
 * followed by the flip; this call exists for per-kernel timing. */
int rbffd_half(const rbffd_plan* plan, const rbffd_fields* f, int32_t which, void* stream);
/* rbffd_run: the forward workload with sources, receivers, energy,
 * checkpoints, optional HIP-graph replay.  workspace: workspace_bytes. */
int rbffd_run(const rbffd_plan* plan, rbffd_fields* f, const rbffd_run_args* args,
              void* workspace, void* stream);
/* rbffd_adjoint: gradients of J(traces) (see rbffd_adjoint_args). */
int rbffd_adjoint(const rbffd_plan* plan, const rbffd_fields* f, const rbffd_adjoint_args* args,
                  void* stream);

/* ---- hyperviscosity per field and the parameter search (Section 5.1) ------
 * rbffd_set_field_hv (K-field batch): field k uses the hyperviscosity constant
 * c_dev[k] (device double [K], the paper's c), i.e. gamma_k = c_k (-1)^(alpha-1)
 * h^(2 alpha); c_dev = NULL gives every field the plan's c again.  Stays in
 * effect for later steps and runs of the plan.
 *
 * rbffd_hv_scan (K-field batch, K >= 3): the paper picks c by running the
 * problem with several c and watching the relative energy u(t) = U(t)/U(0)
 * of eq. 20, with a bisection on c where a fine sweep is slow (Section 5.1,
 * Figures 5-6); Section 6 accepts c when u stays in [0.99, 1.01].  Here each
 * round runs the K fields from the same state (E0, H0), field k with
 * c_k = lo (hi / lo)^(k / (K - 1)) over the current bracket [lo, hi]
 * (initially [c_lo, c_hi]); c_k is accepted when every sample of u_k (every
 * energy_every steps of T) is finite and in [u_lo, u_hi].  The next bracket is
 * [c_{k*-1}, c_{k*}] around the smallest accepted c_{k*}.  The search stops
 * after `rounds` rounds, or early: status 2 when no candidate of the first
 * round is accepted (later rounds keep the previous bracket), status 1 when
 * c_lo of a round is accepted (the edge lies below the bracket); otherwise
 * status 0.  The field buffers are overwritten; the plan's c is restored
 * at the end.  Synchronises the stream.  workspace: as for rbffd_run. */
typedef struct rbffd_hv_scan_args {
    const void* E0;          /* device [N][fe]: one field, internal order, plan type */
    const void* H0;          /* device [N][fh]                                      */
    double c_lo, c_hi;       /* initial bracket, 0 < c_lo < c_hi                    */
    int32_t rounds;          /* >= 1                                                */
    int32_t T;               /* steps per round, >= 1                               */
    int32_t energy_every;    /* >= 1                                                */
    int32_t reserved;
    double u_lo, u_hi;       /* accepted band of u                                  */
    double* c_dev;           /* device scratch [K]                                  */
    double* energy_dev;      /* device scratch [(T-1)/energy_every + 1][K]          */
    double* c_host;          /* host out [rounds][K] candidates (or NULL)           */
    double* umin_host;       /* host out [rounds][K] min of u (or NULL)             */
    double* umax_host;       /* host out [rounds][K] max of u, +inf if not finite   */
    int32_t* ok_host;        /* host out [rounds][K] 1 = accepted (or NULL)         */
    double c_best;           /* out: smallest accepted c, 0 if none                 */
    double bracket[2];       /* out: final bracket                                  */
    int32_t rounds_done;     /* out: rounds run (rows written)                      */
    int32_t status;          /* out: 0 bracketed, 1 edge below c_lo, 2 none         */
} rbffd_hv_scan_args;
int rbffd_set_field_hv(rbffd_plan* plan, const double* c_dev, void* stream);
int rbffd_hv_scan(rbffd_plan* plan, rbffd_fields* f, rbffd_hv_scan_args* args, void* workspace,
                  void* stream);

/* ---- FP64 reductions (eq. 20, eq. 23) -------------------------------------
 * rbffd_energy: out[0] = h^d sum |E|^2 + eta0^2 h_H^d sum |(H_a + H_b)/2|^2
 * for the E buffer E and H buffers Ha, Hb (device double out; workspace as
 * for rbffd_run).
 * rbffd_compare: per component c of a field buffer (which = 0 E, 1 H) in the
 * plan's field layout against ref [N][ncomp] doubles (internal order):
 * out[3c + 0] = sum (f - r)^2, out[3c + 1] = sum r^2, out[3c + 2] = max |f - r|. */
int rbffd_energy(const rbffd_plan* plan, const void* E, const void* Ha, const void* Hb,
                 double* out, void* workspace, void* stream);
int rbffd_compare(const rbffd_plan* plan, int32_t which, const void* field, const double* ref,
                  double* out, void* workspace, void* stream);
/* rbffd_energy_static: rbffd_energy without a workspace argument and without
 * any allocation, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments and result as rbffd_energy (the same kernels, so the same
 * bits).  Its scratch -- the FP64 partial sums of at most 1024 reduction
 * blocks, 8 KB -- is a device array inside the library, one per GPU, held
 * until the process ends; the node count is not limited by it.  Calls that
 * overlap on one GPU share that array and race: serialise them (one stream,
 * or events).  Errors as rbffd_energy; RBFFD_EHIP if the array's address
 * cannot be obtained on the stream's device. */
int rbffd_energy_static(const rbffd_plan* plan, const void* E, const void* Ha, const void* Hb,
                        double* out, void* stream);

/* ---- launch tuning ---------------------------------------------------------
 * Times the step kernels' launch variants on the current device with the
 * given fields (their contents are overwritten) and keeps the fastest in the
 * plan; reps = timed repetitions per variant.  Optional: plans start with a
 * default that is valid everywhere. */
int rbffd_autotune(rbffd_plan* plan, rbffd_fields* f, int32_t reps, void* stream);
/* rbffd_autotune through a cache file of tuned variants, for callers that
 * build plans of the same shape again (serving loops, repeated jobs).  The
 * key is the device (architecture, compute-unit count) and the plan's shape
 * (dimension, node counts, stencil sizes, K, field and weight precision,
 * mode, polarisation, boundary, longest halo list).  Hit: the cached variant
 * is set, nothing runs and f is left as it is (*hit = 1).  Miss: as
 * rbffd_autotune (f advanced by the trial steps), then one line
 * "rbffd-variant <key> <block> <xcd> <lds> <persist>" is appended to
 * cache_path (created if absent; *hit = 0).  Lines that do not parse, and
 * cached variants rbffd_set_variant refuses, are ignored; the last line for
 * a key wins.  hit may be NULL.  RBFFD_EINVAL for a null argument or a file
 * that cannot be written; concurrent writers may interleave lines, which
 * the reader then ignores. */
int rbffd_autotune_cached(rbffd_plan* plan, rbffd_fields* f, int32_t reps, const char* cache_path, int32_t* hit,
                          void* stream);
/* Active launch variant of the step kernels, packed as block | xcd << 16 |
 * lds << 17 | persist << 20 (block = threads per workgroup of the unstaged
 * kernels, xcd = XCD-aware workgroup order, lds = 0 global gathers, 1 LDS-staged
 * kernels when the plan has halo lists, 2 the same but in 3D one staged operand
 * at a time even where both fit, and for the K-field batch persistent staged
 * kernels whose staging wavefronts fill a second LDS buffer while the others
 * sum, 3 in 2D (single field, collocated) global
 * gathers with four wavefronts per 64-node tile, each summing a quarter of the
 * stencil (for node sets too small to fill the chip), persist = resident
 * workgroups per CU of the K-field batch's global kernels and the field-slice
 * width of its staged ones: 16 fields for persist >= 16 where two
 * workgroups' slices fit one CU's LDS, 4 below 8, else 8, each where K and
 * the LDS allow; batch plans start at persist = 16).  rbffd_set_variant sets
 * it (block a multiple of 64, <= 512, lds 0..3). */
int rbffd_get_variant(const rbffd_plan* plan, int32_t* out_variant);
int rbffd_set_variant(rbffd_plan* plan, int32_t block, int32_t xcd, int32_t lds, int32_t persist);

/* ---- measurement ------------------------------------------------------------
 * rbffd_stream_copy: dst[0 .. bytes) = src[0 .. bytes) on the stream with 16-byte
 * non-temporal accesses (device pointers, 16-byte aligned, bytes a multiple of
 * 16; the ranges must not overlap).  Timing it gives the practical HBM
 * ceiling (2 * bytes moved) that the step kernels are compared with. */
int rbffd_stream_copy(const void* src, void* dst, int64_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RBFFD_H */
