// Internal declarations of libl0l2 (host side).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/l0l2.h"

namespace l0l2 {

constexpr int kPadRows = 128;   // n and p are padded to multiples of this
constexpr int kPadNodes = 32;   // K is padded to multiples of this (one GEMM tile)

// Device scratch of the allocation-free entry point (l0l2_refine_incumbent_noalloc):
// its size, and the device indices it serves.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
constexpr int kNoAllocMaxDevices = 64;

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// Leading dimension of a matrix whose rows (or columns) hold `extent` elements
// of `elem` bytes: the extent plus 64 bytes.  The contraction tiles load a
// fragment as 64-byte pieces of 16 consecutive rows; with rows a whole number
// of 128-byte lines apart those loads took up to 35 % longer than with rows
// offset by half a line (measured at n = p = 1024 and 5120 and at p = 50048,
// FP32 and FP64).
inline int64_t ld_pad(int64_t extent, int64_t elem) { return extent + 64 / elem; }

// Error carrying a status code; caught at the C ABI boundary.
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void hip_check(hipError_t e, const char *what);
#define HIPCHK(x) ::l0l2::hip_check((x), #x)

// Device bytes the library holds: process-wide, and per context (charged to the
// context whose call allocated the buffer: the calling thread's current context).
struct MemCount {
    std::atomic<size_t> in_use{0}, peak{0};
    void add(size_t b) {
        const size_t now = in_use.fetch_add(b) + b;
        size_t pk = peak.load();
        while (now > pk && !peak.compare_exchange_weak(pk, now)) {
        }
    }
    void sub(size_t b) { in_use.fetch_sub(b); }
};
MemCount &global_mem();
// The context whose entry point runs on this thread (null outside calls).
MemCount *&thread_mem();

// Device buffer owned by the library.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    MemCount *charged = nullptr;   // the context counter the allocation was charged to
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release();
    // grow to at least `b` bytes (contents not preserved)
    void ensure(size_t b);
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Scalars of the closed forms, evaluated once per instance with the same
// expressions in every precision (the float copies are rounded from these).
struct MethodParams {
    double l0, l2, M, rho;
    double s;           // sqrt(l0 / l2)
    int free_quad;      // s <= M: free coordinates use the 3-piece psi
    double a;           // 2 sqrt(l0 l2) / rho
    double a_plus_s;    // a + s
    double ridge;       // rho / (rho + 2 l2)
    double thr_lin;     // l0 / (M rho) + l2 M / rho
    double thr_free;    // a if free_quad else thr_lin
    double thr_free_M;  // thr_free + M
    double two_M_l2;    // 2 M l2
    double four_l2;     // 4 l2
    double l2_M2;       // l2 M M
    double psi_lin;     // 2 sqrt(l0 l2) if free_quad else l0 / M + l2 M
};

// Tile shapes (index into the sweep kernels' shape table) of the two contractions.
struct TileChoice {
    int xw = 0, xtu = 0;
    int z2 = -1;   // FP64 tiles of reduced modes: the anchor's product over n (-1: not timed)
};

struct Instance {
    int64_t n = 0, p = 0, np = 0, pp = 0;   // true and padded sizes
    // leading dimensions (elements, ld_pad of the padded extents)
    int64_t ldx = 0;    // FP64 column-major X64 and FP64 Xh / Xh64 (np + 8)
    int64_t ldxr = 0;   // FP64 row-major X64R, XhRw (FP64 mode), Xh64R (pp + 8)
    int64_t ldw = 0;    // working-precision column-major Xh / XhLo (FP32 np + 16, BF16 np + 32)
    int64_t ldwr = 0;   // working-precision row-major XhRw / XhR / XhRLo (FP32 pp + 16, BF16 pp + 32)
    int64_t ldp = 0;    // node-state rows (W, beta, V, B, codes and the FP64 copies): pp + 64 bytes of the state type
    int64_t ldu = 0;    // rows of the ADMM product U in the state type (np + 64 bytes)
    int64_t ldu64 = 0;  // rows of the FP64 U64 and of the residuals R (np + 8)
    int prec = L0L2_FP64;
    MethodParams mp{};
    double yy = 0.0;                         // ||y||^2
    DevBuf X64;       // np x pp column-major FP64 (ld ldx), zero padded
    DevBuf y64;       // np
    DevBuf c64;       // ldp, X^T y (zero past p)
    DevBuf colnrm;    // ldp, ||X_j||
    DevBuf cst;       // ldp, c in state precision
    DevBuf Xh;        // np x pp column-major, L^{-1} X in working precision (f64: ld ldx, f32: ld ldw); BF16 mode: high half (ld ldw)
    DevBuf XhLo;      // BF16 mode: column-major low half (Xh - bf16(Xh)), ld ldw
    DevBuf XhR;       // BF16 mode: row-major high half (row i contiguous over pp), ld ldwr
    DevBuf XhRLo;     // BF16 mode: row-major low half, ld ldwr
    DevBuf Xh64;      // FP32 / BF16 mode: FP64 folded operand of the anchored sweeps (ld ldx)
    DevBuf XhRw;      // FP64 / FP32 mode: row-major copy of Xh in the working precision (ld ldxr / ldwr)
    DevBuf Xh64R;     // FP32 / BF16 mode: row-major copy of Xh64 (ld ldxr)
    DevBuf X64R;      // row-major copy of X64 (contraction over p of the gap check), ld ldxr
    DevBuf qR, qC;    // FP8 mode: e4m3 codes of Xh / s (row-major, ld ldqr bytes; column-major, ld ldqc bytes)
    DevBuf qs;        // FP8 mode: FP32 column scales s_j (ldp entries, zero past p)
    int64_t ldqr = 0, ldqc = 0;
    DevBuf codes_pad; // scratch
    std::map<std::pair<int, int64_t>, TileChoice> tiles;   // autotuned per (type, padded K)
    int tuned_K = 0;                                      // node-batch size chosen by measurement (0: none yet)
    // Gram form of the b-update (FP32 mode): G = Xh^T Xh (pp x pp, symmetric),
    // b = (w - G w) / rho in one contraction; built on first use
    DevBuf G64, G32, Ghi, Glo;   // Ghi / Glo: BF16 mode, G as two BF16 terms (ld ldgb)
    int64_t ldg64 = 0, ldg32 = 0, ldgb = 0;
    bool gram_built = false;
    int form_pick = 0;           // b-update form measured on the first solve: 0 not yet, 1 folded, 2 Gram
    double form_ms[2] = {0, 0};  // the per-sweep times that decided it (folded, Gram)
};

// Per-batch workspace, grown on demand (capacity in padded nodes).
struct Workspace {
    int64_t cap = 0;
    DevBuf W, beta, V, B;          // Kp rows of ldp, state precision
    DevBuf W2;                     // FP32 mode: second W (or d) buffer of the Gram-form sweeps
    DevBuf U;                      // Kp rows of ldu, state precision (ADMM product)
    DevBuf Upart;                  // partial products of the contraction over p cut into slices
    DevBuf W64, beta64, V64, B64;  // FP32 / BF16 mode: FP64 state of the anchored sweeps (Kp rows of ldp)
    DevBuf U64;                    // FP32 / BF16 mode: Kp rows of ldu64
    DevBuf Wa, Za;                 // FP32 / BF16 mode: anchor w_a and Xh^T Xh w_a (Kp rows of ldp, FP64)
    DevBuf Wa32, Za32;             // BF16 mode: FP32 anchor of a block of single-term Gram sweeps (Kp rows of ldp)
    DevBuf Dbf[2];                 // BF16 mode: BF16 operand d = W - w_a of the single-term sweeps, alternating
    DevBuf R;                      // Kp rows of ldu64: FP64 residuals of the gap check
    DevBuf codes;                  // Kp rows of ldp, uint8
    DevBuf rpart;                  // Kp x (np/32) x 4 doubles: row-tile sums of the gap check
    DevBuf part;                   // Kp x (pp/32) x 3 doubles
    DevBuf gpart;                  // Kp x (pp/16) x 5 doubles: per-tile sums of the gap estimate
    DevBuf gate;                   // int32: length of the check list
    DevBuf needs;                  // Kp int32: the gap estimate leaves the node to the exact check
    DevBuf gest;                   // Kp FP64: the gap estimate (a lower bound of the exact relative gap)
    DevBuf clist;                  // Kp int32: node slots the exact check evaluates, then -1
    DevBuf list;                   // Kp int32: active node slots of the batch, then -1
    DevBuf nlist, ncount;          // the active list being rebuilt by the check
    DevBuf active, iters, status;  // Kp int32
    DevBuf lb, primal;             // Kp doubles
    DevBuf counter;                // int32 x 3: active nodes, active nodes above the switch tolerance, retired
    DevBuf start;                  // Kp int32: sweep number at which the slot's node started
    DevBuf dlist;                  // Kp int32: slots retired in the last block (counter[2] of them)
    int64_t stat_blocks = 0, stat_sparse = 0, stat_node_blocks = 0;   // blocks of the last solve; with < 1/8 live
    DevBuf sweep_no;               // int32 sweep counter of the batch
    int64_t gen = 0;               // bumped whenever the buffers above move
    DevBuf fista;                  // FP64 residual scratch for the incumbent kernels
    DevBuf fista_wide, fista_list; // slots and node list of supports wider than one workgroup's LDS
    DevBuf nfree;                  // int32 per node: free-coordinate counts of l0l2_round_branch
    DevBuf root_beta, root_v;      // the last branch and bound's root iterates (ldp state elements each)
    bool have_root = false;
    int *host_counter = nullptr;   // pinned
};

enum { PROF_GEMM_XW_F32 = 0, PROF_ADMM_XTU_F32, PROF_GEMM_XW_F64, PROF_ADMM_XTU_F64, PROF_GEMM_XW_BF16,
       PROF_ADMM_XTU_BF16, PROF_CHECK, PROF_ROUND, PROF_FISTA, PROF_ANCHOR, PROF_GEMM_XW_FP8, PROF_ADMM_XTU_FP8,
       kProfCount };
extern const char *const kProfNames[kProfCount];

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t next = 0;
    std::vector<std::pair<int, hipEvent_t>> open;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pairs;
    double total_ms[kProfCount] = {};
    int64_t count[kProfCount] = {};
    int64_t units[kProfCount] = {};   // work units (active node-iterations for the sweeps)
};

// A captured block of sweeps + gap check.
struct GraphKey {
    int kind;
    int64_t Kp, cols;
    int n;
    int force;
    double tol, switch_tol;
    int64_t gen;
    int budget;
    bool operator<(const GraphKey &o) const {
        if (kind != o.kind) return kind < o.kind;
        if (Kp != o.Kp) return Kp < o.Kp;
        if (cols != o.cols) return cols < o.cols;
        if (n != o.n) return n < o.n;
        if (force != o.force) return force < o.force;
        if (tol != o.tol) return tol < o.tol;
        if (switch_tol != o.switch_tol) return switch_tol < o.switch_tol;
        if (gen != o.gen) return gen < o.gen;
        return budget < o.budget;
    }
};

}  // namespace l0l2

namespace l0l2 {
// Executor of blocks of several contexts in shared launches (admm.hip).
struct GroupExec;
struct GroupStats {
    int64_t rounds = 0;     // executor rounds (each runs every block waiting at its start)
    int64_t blocks = 0;     // blocks run
    int64_t launches = 0;   // grouped contraction launches
    int64_t members = 0;    // member contractions in them
};
GroupExec *group_exec_create(int device);
void group_exec_destroy(GroupExec *ex);
// Contexts whose blocks the executor may wait for (+1 when one is attached, -1 when it leaves).
void group_exec_attach(GroupExec *ex, int delta);
GroupStats group_exec_stats(GroupExec *ex);
}  // namespace l0l2

struct l0l2_ctx {
    int device = 0;
    hipStream_t stream = nullptr;       // the context's own stream (non-blocking, default priority)
    hipStream_t user_stream = nullptr;  // the caller's stream, ordered with `stream` by events
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::string err;
    bool has_data = false;
    bool tune = true;          // time the tile shapes of each new batch size
    int force_xw = -1, force_xtu = -1;   // fixed tile shapes (-1: autotune)
    int bform = 0;                       // b-update form: 0 auto, 1 folded operand (two contractions), 2 Gram
    int bf16_terms = 1;                  // BF16 Gram sweeps: 1 single-term anchored blocks, 3 split every sweep
    int bf16_rows = 128;                 // rows of the single-term sweep's largest LDS-staged tile (128 or 256)
    bool use_graphs = true;              // replay captured blocks of sweeps
    std::string noalloc_err;             // why the allocation-free scratch is unavailable (empty: it is)
    std::atomic<int> cancel{0};          // set by l0l2_cancel (any thread), taken by the next block boundary
    l0l2::GroupExec *group = nullptr;    // the executor its blocks go through (server contexts), or none
    hipEvent_t ev_group = nullptr;       // orders the executor's stream after this context's stream
    l0l2::MemCount mem;                  // device bytes held by buffers this context's calls allocated
    std::map<l0l2::GraphKey, hipGraphExec_t> graphs;
    // declared after mem: destroyed before it, so their releases can uncharge it
    l0l2::Instance inst;
    l0l2::Workspace ws;
    l0l2::Profiler prof;
};

namespace l0l2 {

// Throws L0L2_E_CANCELLED (and clears the request) when l0l2_cancel was called
// on ctx; called at block and batch boundaries of the long-running calls.
inline void check_cancel(l0l2_ctx *ctx) {
    if (ctx->cancel.exchange(0) != 0) fail(L0L2_E_CANCELLED, "cancelled by l0l2_cancel");
}

// precompute.hip
void set_data(l0l2_ctx *ctx, const double *X, const double *y, int64_t n, int64_t p, double l0,
              double l2, double M, double rho, int prec, int on_device);
MethodParams make_params(double l0, double l2, double M, double rho);
// New penalties for the loaded instance; the precompute is kept.
void set_penalties(l0l2_ctx *ctx, double l0, double l2, double M);
// max_j of the gain of adding j to the empty support at lambda0 = 0 (App. A.2).
double lambda0_max(l0l2_ctx *ctx);

// admm.hip
void ensure_workspace(l0l2_ctx *ctx, int64_t K);
void load_batch(l0l2_ctx *ctx, int K, const uint8_t *codes, const void *beta, const void *v,
                bool codes_on_host);
void store_batch(l0l2_ctx *ctx, int K, void *beta, void *v, void *b);
void run_sweeps(l0l2_ctx *ctx, int K, int sweeps, bool store_b_last);
void run_dual_bound(l0l2_ctx *ctx, int K, const void *b_internal_or_null);
// Solve the K nodes loaded in the workspace; results stay in ws.lb/primal/iters/status.
void run_solve(l0l2_ctx *ctx, int K, const l0l2_admm_opts &o);
// N queued nodes (device codes N x p, warm starts / results N x p in the state
// type: FP64, or FP32 in the reduced modes) through K slots with refill; results
// to the device arrays lb, primal, iters, status (N each).
void run_queue(l0l2_ctx *ctx, int N, const uint8_t *codes, void *beta, void *v, int K, const l0l2_admm_opts &o,
               double *lb, double *primal, int32_t *iters, int32_t *status);
// Node-batch size by measurement: candidates 32, 64, ... up to k_max; returns
// the chosen K and fills rates[i] (node-sweeps per second of candidate 32 * 2^i).
int tune_batch_size(l0l2_ctx *ctx, int k_max, double frac, std::vector<double> &rates);

// incumbent.hip
void run_round_branch(l0l2_ctx *ctx, int K, const uint8_t *codes, int64_t ld_codes, const void *beta, int64_t ld_beta,
                      uint8_t *support, int32_t *support_size, int32_t *branch_j, int32_t *z_up,
                      int32_t *nfree);
void run_fista(l0l2_ctx *ctx, int K, const uint8_t *support, int64_t ld_support, double *beta,
               int64_t ld_beta, const l0l2_fista_opts &o, double *obj, int32_t *iters, double *resbuf = nullptr);
// Device address of the allocation-free entry point's scratch on `device`
// (which must be current), looked up once per device.
void *noalloc_scratch(int device);
double run_exact_objective(l0l2_ctx *ctx, const uint8_t *support_host, double *beta_host);
// state (f32 or f64, ld_src) -> f64 (ld_dst) copy of K rows of length p
void state_to_f64(l0l2_ctx *ctx, int K, const void *src, int64_t ld_src, double *dst, int64_t ld_dst);

// b-update form (l0l2_bupdate_form): 1 folded, 2 Gram; times of one sweep of
// each as measured (0 when not measured).
int bupdate_form(l0l2_ctx *ctx, double ms[2]);

// heuristic.hip: forward / backward matching pursuit from the empty support;
// host outputs mask and beta (p entries), moves (room for max_moves, may be null)
void run_matching_pursuit(l0l2_ctx *ctx, int max_moves, uint8_t *mask_host, double *beta_host, int32_t *moves_host,
                          int32_t *n_moves, double *obj);

// bnb.hip
void bnb_solve(l0l2_ctx *ctx, const l0l2_bnb_opts &o, l0l2_bnb_result *out);

void drop_graphs(l0l2_ctx *ctx);

// prof.hip
void prof_begin(l0l2_ctx *ctx, int id);
void prof_end(l0l2_ctx *ctx, int id, int64_t units = 0);
void prof_collect(l0l2_ctx *ctx);
void prof_release(Profiler &p);

inline size_t state_bytes(int prec) { return prec == L0L2_FP64 ? 8 : 4; }

}  // namespace l0l2
