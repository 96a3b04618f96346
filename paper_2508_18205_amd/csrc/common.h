// Internal definitions shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/rbffd.h"

#define RBFFD_MAX_STENCIL 128     // max(n, n_hv) supported
#define RBFFD_MAX_MONO 64         // monomials per local system
#define RBFFD_TILE 64             // nodes per packed tile (one wavefront)
#define RBFFD_WGT 256             // nodes per LDS-staged workgroup tile (4 wavefronts)
#define RBFFD_WGT_BATCH 128       // K-field batch: nodes per staged tile (two workgroups share a CU)
#define RBFFD_WGT_3D 512          // 3D: nodes per staged workgroup tile (8 wavefronts)
#define RBFFD_WGT_3D_F32 1024     // 3D with FP32 fields (16 wavefronts)
#define RBFFD_LDS_BUDGET 65536    // bytes of LDS one staged workgroup may use
#define RBFFD_LDS_BUDGET_3D 131072 // 3D: both operands together up to this size (one
                                   // workgroup per CU; the tuner also tries one operand
                                   // at a time, two per CU)
#define RBFFD_KSLICE 16           // widest field slice of the staged K-field batch
#define RBFFD_LDS_BUDGET_BATCH 122880
#define RBFFD_LDS_CU 163840       // LDS of one CU (gfx950)

// ---------------------------------------------------------------------------
// Device-side layout of one operator block (the weights applied in one half
// step).  Packed arrays are "tile-sliced ELL": node i = 64 t + l lives in tile
// t, lane l; slot chunk q (4 consecutive non-self slots) of tile t occupies a
// contiguous run of 64 x 4 values, so one wavefront streams 1 KB (FP32) per
// load instruction.  Difference form: the slot whose value is used as
// reference (the node itself for collocated stencils) is not stored; since
// every weight vector sums to zero (constants are reproduced), sum_s w_s f_s
// = sum_{s != ref} w_s (f_s - f_ref).
// ---------------------------------------------------------------------------
struct OpBlock {
    int64_t Nt = 0;          // target (centre) nodes
    int64_t Ns = 0;          // source nodes
    int32_t n = 0, nh = 0;   // curl / HV stencil sizes
    int32_t ns = 0;          // union width (collocated) else 0
    bool cross = false;      // curl stencil drawn from the other set (two-set)
    int64_t tiles = 0;
    int32_t C4 = 0, V4 = 0, S4 = 0;  // slot chunks: curl, hv, union index
    // device pointers (inside the arena)
    int32_t* st_union = nullptr;   // [Nt][ns]          (collocated)
    int32_t* st_curl = nullptr;    // [Nt][n]           (two-set)
    int32_t* st_hv = nullptr;      // [Nt][nh]          (two-set)
    double* wc = nullptr;          // [Nt][dim][n]
    double* wh = nullptr;          // [Nt][nh]
    void* pidx = nullptr;          // collocated: [tiles][S4][64][4] i32 ; two-set: curl chunks
    void* pidx_h = nullptr;        // two-set: [tiles][V4][64][4] i32 hv chunks
    int32_t* pref = nullptr;       // two-set: [Nt] reference (slot 0) of the curl stencil
    void* pwc = nullptr;           // [tiles][C4][dim][64][4] weights
    void* pwh = nullptr;           // [tiles][V4][64][4] weights
    // node-major copies for the K-field batch (collocated only)
    int32_t* bidx = nullptr;       // [Nt][S4*4]
    float* bwc = nullptr;          // [Nt][dim][C4*4]
    float* bwh = nullptr;          // [Nt][V4*4]
    float* bw0 = nullptr;          // [Nt][4]: centre weights (curl x, curl y, hyperviscosity, 0)
    // LDS staging (collocated): per 256-node workgroup tile, the sorted unique
    // source nodes of all its stencils ("halo list") and, per node and slot,
    // the 16-bit position of the slot's node in that list
    uint16_t* lidx = nullptr;      // [tiles][Q8][64][8]
    uint16_t* lself = nullptr;     // [tiles * 64] each node's own position (K-field batch)
    int32_t* hpool = nullptr;      // concatenated halo lists
    int32_t* hoff = nullptr;       // [nwg + 1] start of each workgroup's list
    int32_t Q8 = 0;
    int64_t nwg = 0;
    int32_t wgt = RBFFD_WGT;       // nodes per staged workgroup tile (halo lists)
    int32_t hmax = 0;              // longest halo list (0 = staging unavailable)
    int32_t stage = 0;             // single field: 1 = both operands staged together,
                                   // 2 = one operand at a time (3D), 0 = none
    // transposed operator for the adjoint (collocated 2D)
    int64_t* t_off = nullptr;      // [tiles + 1] start of each tile's entries
    int32_t* t_width = nullptr;    // [tiles]
    int32_t* t_src = nullptr;      // [entries]  source row i
    int32_t* t_slot = nullptr;     // [entries]  slot s of row i (-1 = padding)
    void* t_w = nullptr;           // [entries][4] (wx, wy, wh, 0) in weight precision
    int64_t t_cap = 0;             // entry capacity
};

struct NodeSet {
    int64_t N = 0;
    std::vector<double> xyz_host;
    std::vector<uint8_t> flags_host;
    double* xyz_in = nullptr;     // [N][dim] original order
    uint8_t* flags_in = nullptr;  // [N]
    int32_t* perm = nullptr;      // internal -> original
    int32_t* inv = nullptr;       // original -> internal
    double* xyz = nullptr;        // [N][dim] internal order
    uint8_t* emask = nullptr;     // [N] bit c = E component c free (E set only);
                                  // bit 3 = curved wall with a normal in nrm
    std::vector<double> nrm_host; // [N][dim] unit wall normals, original order
    double* nrm = nullptr;        // [N][dim] internal order (see has_wall_normals)
    double h = 0;
};

struct Variant {
    int block = 256;      // threads per workgroup (multiple of 64)
    int xcd = 1;          // XCD-aware block remap
    int persist = 8;      // K-field batch: resident workgroups per CU
    int lds = 1;          // use the LDS-staged step kernels when available
};

struct rbffd_plan {
    rbffd_params p{};
    int dim = 2;
    int n = 0, nh = 0, ns = 0;
    int M = 0, Mh = 0;
    int FE = 1, FH = 2;          // stored values per node
    int fe_comp = 1, fh_comp = 2;// physical components
    int K = 1;
    double dt = 0, gamma = 0, c0 = 1, eta0 = 1;
    double hv_fac = 0;           // gamma / c = (-1)^(alpha-1) h^(2 alpha)
    float* gk = nullptr;         // K-field batch: per-field gamma [K] (arena)
    NodeSet E, H;                // H unused unless two-set
    OpBlock opH, opE;            // operators of the H update and the E update
    bool collocated = true;
    // arena / workspace bookkeeping
    int64_t arena_bytes = 0, ws_bytes = 0, adj_ws_bytes = 0;
    int64_t t_entries = 0;       // entries of the transposed operator
    char* arena = nullptr;
    bool ready = false;
    Variant var;
    // private stream used only to capture HIP graphs (the caller's stream may
    // be the legacy null stream, which cannot be captured); default priority
    mutable hipStream_t cap_stream = nullptr;
    std::string err;
    // Morton quantisation box (square): lo and common side
    double mlo[3] = {0, 0, 0};
    double mside = 1;
    int ex_m[RBFFD_MAX_MONO][3];   // monomial exponents (curl)
    int ex_h[RBFFD_MAX_MONO][3];   // monomial exponents (hv)
};

// Plans whose PEC walls may be curved keep per-node wall normals: where E is
// a vector (TEz, 3D) and the walls are PEC.
inline bool has_wall_normals(const rbffd_plan* p) {
    return p->p.bc == RBFFD_BC_PEC && (p->p.pol == RBFFD_POL_TE || p->dim == 3);
}

// ---- run workspace: FP64 reduction partials, the device step counter -------
constexpr int RED_BLOCKS = 1024;
struct RunWS {
    double* part;       // [RED_BLOCKS * 12]
    int32_t* ctr;
    double* misc;
};
inline RunWS run_ws(void* ws) {
    RunWS w;
    char* b = (char*)ws;
    w.part = (double*)b;
    w.ctr = (int32_t*)(b + RED_BLOCKS * 12 * 8);
    w.misc = (double*)(b + RED_BLOCKS * 12 * 8 + 256);
    return w;
}

// K-field batch: per-field gamma from per-field constants c (device [K]), or
// every field the plan's gamma when c is null (batched.hip)
int fill_field_gamma(const rbffd_plan* p, const double* c_dev, hipStream_t st);

// ---- helpers --------------------------------------------------------------
int set_err(const rbffd_plan* p, int code, const std::string& msg);
#define HIPCHK(plan, call)                                                       \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess)                                                    \
            return set_err(plan, RBFFD_EHIP, std::string(#call) + ": " +         \
                                                 hipGetErrorString(e_));         \
    } while (0)

static inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

int64_t n_monomials(int d, int m);
void fill_exponents(int d, int m, int ex[RBFFD_MAX_MONO][3]);
int field_elem_bytes(int fdtype);
int weight_elem_bytes(int wdtype);

// layout: assigns offsets (when base != nullptr also the pointers); returns
// arena bytes; ws receives the workspace requirement
int64_t layout_arena(rbffd_plan* p, char* base, int64_t* ws, int64_t* adj_ws);

// set-up entry points (setup.hip)
int setup_nodes_and_stencils(rbffd_plan* p, void* ws, hipStream_t s);
int setup_weights(rbffd_plan* p, void* ws, hipStream_t s);
int pack_all(rbffd_plan* p, void* ws, hipStream_t s);
int build_transpose(rbffd_plan* p, void* ws, hipStream_t s);
int refill_transpose(rbffd_plan* p, hipStream_t s);
int build_halos(rbffd_plan* p, void* ws, hipStream_t s);
int64_t setup_ws_bytes(const rbffd_plan* p);
int capture_stream(const rbffd_plan* p, hipStream_t* out);

// ---- HIP-graph step loop -----------------------------------------------------
// The step loop of rbffd_run is replayed from HIP graphs: one graph of S
// captured steps (S even, at most RBFFD_GRAPH_STEPS) replayed T / S times,
// then one graph of the remaining whole step pairs.  rec(c, stream) records
// one full step reading buffer set c; the buffers alternate within a graph
// and, S being even, every replay leaves them as it found them.  *done
// receives the number of steps replayed (even); the caller runs the rest.
#define RBFFD_GRAPH_STEPS 64
template <typename Rec>
int replay_steps(const rbffd_plan* p, int T, int cur, hipStream_t st, Rec rec, int* done) {
    *done = 0;
    if (T < 4) return RBFFD_OK;
    hipStream_t cs;
    int rc = capture_stream(p, &cs);
    if (rc) return rc;
    int left = T;
    while (left >= 4) {
        const int S = std::min(left & ~1, RBFFD_GRAPH_STEPS);
        hipGraph_t g;
        hipGraphExec_t ge;
        HIPCHK(p, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < S; ++k) rec((cur + k) & 1, cs);
        HIPCHK(p, hipStreamEndCapture(cs, &g));
        HIPCHK(p, hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        const int reps = left / S;
        for (int r = 0; r < reps; ++r) HIPCHK(p, hipGraphLaunch(ge, st));
        HIPCHK(p, hipGraphExecDestroy(ge));
        HIPCHK(p, hipGraphDestroy(g));
        left -= reps * S;
        *done += reps * S;
    }
    return RBFFD_OK;
}

// XCD-aware mapping of a linear workgroup id: consecutive logical ids land on
// the same XCD (round-robin dispatch sends block b to XCD b % 8), so
// spatially adjacent tiles share one L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int x = b & 7, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}
