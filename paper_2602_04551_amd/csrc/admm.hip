// Batched ADMM for the node relaxations (Sec. 3.1 and 3.2).
//
// One sweep over K nodes, in the folded Woodbury form with Xh = L^{-1} X:
//   W  = c + rho beta - V                       (formed by the previous epilogue)
//   U  = Xh W^T                 (n x K)        contraction over p   [k_gemm_xw]
//   Q  = Xh^T U                 (p x K)        contraction over n   [k_admm_xtu]
//   b  = (W - Q^T) / rho        = D w row by row (eq. batched_b_update)
//   beta = prox(b + V / rho)    (eq. minbetalower / batched_beta_update)
//   V  = V + rho (b - beta)     (eq. batched_v_update)
//   W' = c + rho beta - V       for the next sweep
// The prox/V/W update is the epilogue of the second contraction, so the K x p
// state is read and written once per sweep.
//
// Every check_every sweeps the relative gap (P(beta) - LB) / |P(beta)| is
// evaluated in FP64 with the original X (Sec. 3.1.2 and the node stopping rule
// of Sec. 4.1): r = y - X b, g = X^T r, LB = rigorous D(r); P(beta) from X beta.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

#include "device_math.hpp"
#include "internal.hpp"

namespace l0l2 {

namespace {

// f(std::integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time.
template <class F, int... I>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F &&f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

template <class T>
DevParams<T> dev_params(const MethodParams &m) {
    DevParams<T> q;
    q.M = (T)m.M;
    q.rho = (T)m.rho;
    int e = 0;
    // a normal power of two whose reciprocal is normal too
    q.rho_pow2 = std::frexp((double)q.rho, &e) == 0.5 && std::fabs((double)q.rho) >= 4.0 * (double)std::numeric_limits<T>::min() &&
                 std::fabs((double)q.rho) <= 0.25 / (double)std::numeric_limits<T>::min();
    q.inv_rho = q.rho_pow2 ? (T)(1.0 / (double)q.rho) : T(0);
    q.a_plus_s = (T)m.a_plus_s;
    q.ridge = (T)m.ridge;
    q.thr_free = (T)m.thr_free;
    q.thr_free_M = (T)m.thr_free_M;
    q.free_quad = m.free_quad;
    return q;
}

// ---------------------------------------------------------------------------
// batch load / store
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_load_state(const T *__restrict__ src, int64_t K, int64_t p, T *__restrict__ dst, int64_t Kp,
                             int64_t pp) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < Kp * pp; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t k = idx / pp, j = idx % pp;
        dst[idx] = (k < K && j < p) ? src[k * p + j] : T(0);
    }
}

__global__ void k_load_codes(const uint8_t *__restrict__ src, int64_t K, int64_t p, uint8_t *__restrict__ dst,
                             int64_t Kp, int64_t pp) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < Kp * pp; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t k = idx / pp, j = idx % pp;
        dst[idx] = (k < K && j < p) ? src[k * p + j] : (uint8_t)CODE_FIX0;
    }
}

template <class T>
__global__ void k_store_state(const T *__restrict__ src, int64_t K, int64_t p, int64_t pp, T *__restrict__ dst) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < K * p; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t k = idx / p, j = idx % p;
        dst[idx] = src[k * pp + j];
    }
}

// Batch start: nodes 0..K-1 active (the active list is 0..K-1), padding inactive.
__global__ void k_set_active(int *active, int *status, int *iters, int *list, int *clist, int64_t K, int64_t Kp,
                             int *sweep_no, int *start) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < Kp) {
        active[k] = k < K;
        status[k] = 1;
        iters[k] = 0;
        list[k] = k < K ? (int)k : -1;
        clist[k] = -1;
        start[k] = 0;
    }
    if (k == 0) *sweep_no = 0;
}

// Sweep counter of the batch, advanced at the start of each block of sweeps;
// the check list, the next active list and the result counters of the block
// start empty.
__global__ void k_sweep_add(int *sweep_no, int n, int *gate, int *ncount, int *counter) {
    *sweep_no += n;
    gate[0] = 0;
    *ncount = 0;
    counter[0] = 0;
    counter[1] = 0;
    counter[2] = 0;
}

// Warm start of Sec. 3.1.3: impose F0 on beta, then W = c + rho beta - V.
template <class T>
__global__ void k_init(const uint8_t *__restrict__ codes, T *__restrict__ beta, const T *__restrict__ V,
                       T *__restrict__ W, const T *__restrict__ c, T rho, int64_t pp, int64_t total) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t j = idx % pp;
        T b = codes[idx] == CODE_FIX0 ? T(0) : beta[idx];
        beta[idx] = b;
        W[idx] = c[j] + rho * b - V[idx];
    }
}

// ---------------------------------------------------------------------------
// Cross-wave partial sums of a TM x TN output tile in LDS: wave w's element
// (m, n) sits at red[w * WS + n * LD + m] with LD = TM + 1 (the pad element
// spreads the 16 lanes that hold one row of an MFMA block over different banks).
// ---------------------------------------------------------------------------
template <int TM, int TN>
struct Red {
    static constexpr int LD = TM + 1, WS = TN * LD;
};

template <class TC, int TM, int TN, int WAVES>
__device__ __forceinline__ TC sum_waves(const TC *red, int n, int m) {
    const int o = n * Red<TM, TN>::LD + m;
    TC s = red[o];
    for (int w = 1; w < WAVES; ++w) s += red[w * Red<TM, TN>::WS + o];
    return s;
}

// ---------------------------------------------------------------------------
// One TM x TN output tile (TM = 16 BM, TN = 16 BN) of C[m][n] = sum_k A[m][k] B[n][k]
// with A rows (lda) and B rows (ldb) contiguous in k.  Both contractions of a
// sweep have this shape: over p with A = the row-major copy of Xh and B = the
// node operand W; over n with A = Xh column-major (a column of Xh is a row of
// Xh^T) and B = U.  The WAVES waves of the workgroup split the chunks of 16 k
// in pairs (wave w takes pairs [npr w / WAVES, npr (w + 1) / WAVES), npr =
// kdim / 32); lane l loads 4 consecutive k of row l%16 with one vector load per
// fragment and the 4 MFMAs of a chunk map their k slot to those 4 values for
// both operands.  Two register stages: the next chunk's loads are issued before
// the current chunk's MFMAs.  The loop body has no branch and scheduling
// barriers keep each load group ahead of the MFMAs that do not need it, so the
// wait before a chunk's MFMAs covers only that chunk's loads (a conditional
// load, or a load the scheduler sinks below the MFMAs, makes that wait cover
// the next chunk's loads too).  On return red holds every wave's partial sums
// (layout Red<TM, TN>) and the workgroup is synchronised.  kdim must be a
// multiple of 32.
// ---------------------------------------------------------------------------
// Node columns of a launch.  Column c of the grid's node range is node slot
// cols[c]; the list holds the live nodes first and -1 in every entry past them
// (up to the padded batch), so a column is idle when its entry is negative and
// a workgroup whose first column is idle has no live column (its workgroup
// returns at once; an idle column of a live workgroup loads a valid row and
// stores nothing).  cols == nullptr: column c is slot c and every column of the
// grid is live.  Converged nodes thus cost nothing: the list holds the nodes
// still active.  A kernel reads the entries of all its columns first, in one
// round trip, before it loads anything that depends on them.
struct NodeCols {
    const int *cols;
};

__device__ __forceinline__ int col_slot(const NodeCols &nc, int64_t c) { return nc.cols ? nc.cols[c] : (int)c; }
// Row of the node arrays read for a column: its slot, or row c (a valid padded
// row, read but never written) when the column is idle.
__device__ __forceinline__ int64_t col_row(int slot, int64_t c) { return slot >= 0 ? (int64_t)slot : c; }

// Slots of the BN fragment rows of this lane (rows n0 + 16 j + lane % 16) and of
// the E epilogue columns of this thread (thread t owns elements t + i 64 WAVES of
// the TM x TN tile, column = element / TM).  Returns false for an idle tile.
template <int TM, int BN, int E, int WAVES>
__device__ __forceinline__ bool tile_slots(const NodeCols &ncl, int64_t n0, int (&sb)[BN], int (&se)[E]) {
    const int r = threadIdx.x & 15;
#pragma unroll
    for (int j = 0; j < BN; ++j) sb[j] = col_slot(ncl, n0 + 16 * j + r);
#pragma unroll
    for (int t = 0; t < E; ++t) se[t] = col_slot(ncl, n0 + (threadIdx.x + t * 64 * WAVES) / TM);
    // lane 0 holds column n0, the first column of the tile
    return __builtin_amdgcn_readfirstlane(sb[0]) >= 0;
}

template <class TC, int BM, int BN, class TA, class TB>
__device__ __forceinline__ void mma_chunk(typename Acc<TC>::type (&acc)[BM][BN], const TA (&a)[BM][4],
                                          const TB (&b)[BN][4]) {
    for (int t = 0; t < 4; ++t)
        for (int i = 0; i < BM; ++i)
            for (int j = 0; j < BN; ++j) acc[i][j] = mfma16((TC)a[i][t], (TC)b[j][t], acc[i][j]);
}

template <class TA, class TB, class TC, int BM, int BN, int WAVES>
__device__ __forceinline__ void nt_tile(const TA *__restrict__ A, int64_t lda, const TB *__restrict__ B, int64_t ldb,
                                        int64_t kdim, int64_t m0, int64_t n0, const int (&sb)[BN], TC *red,
                                        int64_t pr0 = 0, int64_t pr1 = -1) {
    constexpr int TM = 16 * BM, TN = 16 * BN;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int q = lane >> 4, r = lane & 15;
    typedef typename Acc<TC>::type AccT;
    AccT acc[BM][BN];
    for (int i = 0; i < BM; ++i)
        for (int j = 0; j < BN; ++j) acc[i][j] = AccT{0, 0, 0, 0};
    // pairs [pr0, pr1) of the workgroup (all of kdim by default), split over the waves
    if (pr1 < 0) pr1 = kdim / 32;
    const int64_t npr = pr1 - pr0;
    const int wu = __builtin_amdgcn_readfirstlane(w);
    const int64_t c0 = 2 * (pr0 + npr * wu / WAVES), c1 = 2 * (pr0 + npr * (wu + 1) / WAVES);
    const TA *Ap[BM];
    const TB *Bp[BN];
    for (int i = 0; i < BM; ++i) Ap[i] = A + (m0 + 16 * i + r) * lda + 4 * q;
    for (int j = 0; j < BN; ++j) Bp[j] = B + col_row(sb[j], n0 + 16 * j + r) * ldb + 4 * q;
    TA a0[BM][4], a1[BM][4];
    TB b0[BN][4], b1[BN][4];
#define L0L2_LD(a, b, c)                                                  \
    for (int i = 0; i < BM; ++i) load4(Ap[i] + 16 * (c), a[i]);          \
    for (int j = 0; j < BN; ++j) load4(Bp[j] + 16 * (c), b[j]);          \
    __builtin_amdgcn_sched_barrier(0);
    if (c0 < c1) {
        L0L2_LD(a0, b0, c0)
        int64_t c = c0;
        for (; c + 2 < c1; c += 2) {
            L0L2_LD(a1, b1, c + 1)
            mma_chunk<TC, BM, BN>(acc, a0, b0);
            __builtin_amdgcn_sched_barrier(0);
            L0L2_LD(a0, b0, c + 2)
            mma_chunk<TC, BM, BN>(acc, a1, b1);
            __builtin_amdgcn_sched_barrier(0);
        }
        L0L2_LD(a1, b1, c + 1)
        mma_chunk<TC, BM, BN>(acc, a0, b0);
        mma_chunk<TC, BM, BN>(acc, a1, b1);
    }
#undef L0L2_LD
    for (int i = 0; i < BM; ++i)
        for (int j = 0; j < BN; ++j)
            for (int v = 0; v < 4; ++v) {
                int m = 16 * i + acc_row<TC>(lane, v);
                int n = 16 * j + r;
                red[w * Red<TM, TN>::WS + n * Red<TM, TN>::LD + m] = acc[i][j][v];
            }
    __syncthreads();
}

// Contraction over p: U[k][i] = sum_j Xh[i][j] W[k][j] (A = row-major Xh), for
// the node slots k of the live columns.  With gridDim.z = S > 1 slice z takes
// pairs [npr z / S, npr (z + 1) / S) of the 32-wide pairs of k and writes its
// partial product to U + z pstride (added in slice order by k_splitk_sum): a
// grid of S times as many workgroups for few live nodes and a long range p.
// The workgroup's tile (bx, by) of slice z of S (the grid's coordinates, or a
// grouped launch's tile of one member).
template <class TA, class TB, class TC, int BM, int BN, int WAVES>
__device__ __forceinline__ void xw_tile(const TA *__restrict__ A, int64_t lda, const TB *__restrict__ B, int64_t ldb,
                                        TC *__restrict__ U, int64_t ldu, int64_t kdim, NodeCols ncl, int64_t pstride,
                                        int64_t bx, int64_t by, int64_t z, int64_t S, TC *red) {
    constexpr int TM = 16 * BM, TN = 16 * BN, E = TM * TN / (64 * WAVES);
    static_assert(E * 64 * WAVES == TM * TN, "tile elements per thread");
    const int64_t m0 = bx * TM, n0 = by * TN;
    int sb[BN], se[E];
    if (!tile_slots<TM, BN, E, WAVES>(ncl, n0, sb, se)) return;
    const int64_t npr = kdim / 32;
    U += pstride * z;
    nt_tile<TA, TB, TC, BM, BN, WAVES>(A, lda, B, ldb, kdim, m0, n0, sb, red, npr * z / S, npr * (z + 1) / S);
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * WAVES, n = idx / TM, m = idx % TM;
        if (se[t] >= 0) U[(int64_t)se[t] * ldu + m0 + m] = sum_waves<TC, TM, TN, WAVES>(red, n, m);
    }
}

template <class TA, class TB, class TC, int BM, int BN, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_gemm_xw(const TA *__restrict__ A, int64_t lda,
                                                        const TB *__restrict__ B, int64_t ldb, TC *__restrict__ U,
                                                        int64_t ldu, int64_t kdim, NodeCols ncl, int64_t pstride) {
    __shared__ TC red[WAVES * Red<16 * BM, 16 * BN>::WS];
    xw_tile<TA, TB, TC, BM, BN, WAVES>(A, lda, B, ldb, U, ldu, kdim, ncl, pstride, blockIdx.x, blockIdx.y, blockIdx.z,
                                       gridDim.z, red);
}

// Scalars of the gap estimate (FP64).
struct GateArgs {
    double l0, l2, M, s, two_M_l2, four_l2, l2_M2, psi_lin;
    int free_quad;
};

// Operands of the ADMM update of one (node, coordinate), loaded before the
// contraction so that their latency overlaps it.  on: live column and active node.
template <class T>
struct EpiIn {
    T w, v, c;
    uint8_t code;
    bool on;
};

template <class T>
__device__ __forceinline__ void epi_load(EpiIn<T> &ei, int slot, int64_t col, int64_t j, int64_t ldp,
                                         const T *W, const T *__restrict__ V,
                                         const uint8_t *__restrict__ codes, const T *__restrict__ c,
                                         const int *__restrict__ active) {
    const int64_t row = col_row(slot, col), o = row * ldp + j;
    ei.w = W[o];
    ei.v = V[o];
    ei.c = c[j];
    ei.code = codes[o];
    const int act = active[row];   // loaded unconditionally: no wait before the other loads
    ei.on = (slot >= 0) & (act != 0);
}

// The ADMM update of one (node, coordinate) from Q = (Xh^T Xh w)_j:
//   b = (W - Q) / rho, beta = prox(b + V / rho), V += rho (b - beta),
//   W = c + rho beta - V.
// With est set it also returns the five terms of the gap estimate.  Since b
// solves (X^T X + rho I) b = w, the residual r = y - X b satisfies
// X^T r = c - w + rho b and ||r||^2 = ||y||^2 - 2 c^T b + b^T (w - rho b), so the
// dual value D(r) of Prop. 1 and the lower bound
//   P(beta) >= 1/2 ||r||^2 - (X^T r)^T (beta - b) + sum psi(beta)
// (from ||r - X (beta - b)||^2 >= ||r||^2 - 2 r^T X (beta - b)) follow from the
// per-node sums of c b, b (w - rho b), nu(|X^T r|), (X^T r) (beta - b), psi(beta).
// Returns the new W.
template <class T>
__device__ __forceinline__ T admm_update(T Qv, const EpiIn<T> &ei, int64_t o, T *__restrict__ W,
                                         T *__restrict__ beta, T *__restrict__ V, T *__restrict__ Bst,
                                         const DevParams<T> &q, int store_b, bool est, const GateArgs &ga,
                                         double e[5]) {
    const uint8_t code = ei.code;
    const T wv = ei.w;
    const T bb = div_rho(wv - Qv, q);
    const T v = ei.v;
    const T bt = bb + div_rho(v, q);
    const T be = prox_beta(bt, code, q);
    const T vn = v + q.rho * (bb - be);
    const T cj = ei.c;
    const T wn = cj + q.rho * be - vn;
    V[o] = vn;
    W[o] = wn;
    // beta is read only after a block's last sweep (gap check, promotion,
    // read-back), which is the sweep that stores it, with b
    if (store_b) {
        beta[o] = be;
        Bst[o] = bb;
    }
    if (est) {
        const double b = (double)bb, w = (double)wv, cd = (double)cj, rho = (double)q.rho, bn = (double)be;
        const double g = cd - w + rho * b;
        e[0] = cd * b;
        e[1] = b * (w - rho * b);
        e[2] = nu_plain(fabs(g), code, ga.l0, ga.l2, ga.M, ga.two_M_l2, ga.four_l2, ga.l2_M2, ga.free_quad);
        e[3] = g * (bn - b);
        e[4] = psi_val(bn, code, ga.l0, ga.l2, ga.s, ga.free_quad, ga.psi_lin);
    }
    return wn;
}

// The same with the operands loaded here (LDS-staged tiles, whose lanes own too
// many elements to load them ahead).
template <class T>
__device__ __forceinline__ T admm_update(T Qv, int64_t o, int64_t j, T *__restrict__ W, T *__restrict__ beta,
                                         T *__restrict__ V, T *__restrict__ Bst, const uint8_t *__restrict__ codes,
                                         const T *__restrict__ c, const DevParams<T> &q, int store_b, bool est,
                                         const GateArgs &ga, double e[5]) {
    EpiIn<T> ei;
    ei.w = W[o];
    ei.v = V[o];
    ei.c = c[j];
    ei.code = codes[o];
    ei.on = true;
    return admm_update<T>(Qv, ei, o, W, beta, V, Bst, q, store_b, est, ga, e);
}

// Sums the five estimate terms over the TM consecutive threads that hold one
// node's coordinates of the tile and stores them at gpart[(node * ntile + tile) * 5].
template <int TM>
__device__ __forceinline__ void store_estimate(double e[5], int m, int64_t node, double *__restrict__ gpart,
                                               int64_t ntile, int64_t tile) {
    for (int t = 0; t < 5; ++t)
        for (int off = 1; off < TM; off <<= 1) e[t] += __shfl_xor(e[t], off);
    if (m == 0 && node >= 0) {
        double *d = gpart + (node * ntile + tile) * 5;
        for (int t = 0; t < 5; ++t) d[t] = e[t];
    }
}

// The row tiles of the grid's x axis.
template <int TM>
__device__ __forceinline__ void store_estimate(double e[5], int m, int64_t node, double *__restrict__ gpart) {
    store_estimate<TM>(e, m, node, gpart, (int64_t)gridDim.x, (int64_t)blockIdx.x);
}

// Contraction over n with the ADMM epilogue: Q[k][j] = sum_i Xh[i][j] U[k][i],
// then admm_update for node k and coordinate j, reading W and writing the new W
// to Wout (the same array, or in the Gram form, whose operand U is W itself,
// the other buffer of a pair).  gpart != nullptr adds the per-tile sums of the
// gap estimate.
template <class TA, class T, int BM, int BN, int WAVES>
__device__ __forceinline__ void xtu_tile(const TA *__restrict__ A, int64_t lda, const T *__restrict__ U, int64_t ldu,
                                         int64_t kdim, const T *W, T *Wout, T *__restrict__ beta, T *__restrict__ V,
                                         T *__restrict__ Bst, const uint8_t *__restrict__ codes,
                                         const T *__restrict__ c, const int *__restrict__ active,
                                         const DevParams<T> &q, int64_t ldp, int store_b, double *__restrict__ gpart,
                                         const GateArgs &ga, NodeCols ncl, int64_t bx, int64_t by, int64_t gx, T *red) {
    constexpr int TM = 16 * BM, TN = 16 * BN, E = TM * TN / (64 * WAVES);
    static_assert(E * 64 * WAVES == TM * TN, "tile elements per thread");
    const int64_t m0 = bx * TM, n0 = by * TN;
    int sb[BN], se[E];
    if (!tile_slots<TM, BN, E, WAVES>(ncl, n0, sb, se)) return;
    EpiIn<T> ei[E];
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * WAVES;
        epi_load<T>(ei[t], se[t], n0 + idx / TM, m0 + idx % TM, ldp, W, V, codes, c, active);
    }
    nt_tile<TA, T, T, BM, BN, WAVES>(A, lda, U, ldu, kdim, m0, n0, sb, red);
    const bool est = gpart != nullptr;
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * WAVES, n = idx / TM, m = idx % TM;
        double e[5] = {0, 0, 0, 0, 0};
        if (ei[t].on)
            admm_update<T>(sum_waves<T, TM, TN, WAVES>(red, n, m), ei[t], (int64_t)se[t] * ldp + m0 + m, Wout, beta, V,
                           Bst, q, store_b, est, ga, e);
        if (est) store_estimate<TM>(e, m, se[t], gpart, gx, bx);
    }
}

template <class TA, class T, int BM, int BN, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_admm_xtu(const TA *__restrict__ A, int64_t lda, const T *__restrict__ U,
                                                  int64_t ldu, int64_t kdim, const T *W, T *Wout,
                                                  T *__restrict__ beta, T *__restrict__ V, T *__restrict__ Bst,
                                                  const uint8_t *__restrict__ codes, const T *__restrict__ c,
                                                  const int *__restrict__ active, DevParams<T> q, int64_t ldp,
                                                  int store_b, double *__restrict__ gpart, GateArgs ga, NodeCols ncl) {
    __shared__ T red[WAVES * Red<16 * BM, 16 * BN>::WS];
    xtu_tile<TA, T, BM, BN, WAVES>(A, lda, U, ldu, kdim, W, Wout, beta, V, Bst, codes, c, active, q, ldp, store_b,
                                   gpart, ga, ncl, blockIdx.x, blockIdx.y, gridDim.x, red);
}

// ---------------------------------------------------------------------------
// Anchored FP64 sweeps (FP32 mode, after the reduced-precision phase).  At the
// start of a block the FP64 iterate w_a = W and its product z_a = Xh^T Xh w_a
// are formed in FP64; each sweep then multiplies only the difference
// d = fl32(W - w_a) in FP32 and takes Xh^T Xh W = z_a + Xh^T Xh d, so the
// product's rounding error scales with |d| (the movement within the block)
// rather than with |W|, while the state and the update stay FP64.
// ---------------------------------------------------------------------------
__global__ void k_anchor_init(const double *__restrict__ W, double *__restrict__ Wa, float *__restrict__ d,
                              int64_t total) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        Wa[idx] = W[idx];
        d[idx] = 0.0f;
    }
}

// Contraction over n of an anchored sweep: Q32 = Xh^T U32 (FP32 MFMA), then
// admm_update<double> with Q = z_a + Q32 and d = fl32(W_new - w_a).
template <int BM, int BN, int WAVES>
__device__ __forceinline__ void xtu_anch_tile(
    const float *__restrict__ A, int64_t lda, const float *__restrict__ U, int64_t ldu, int64_t kdim,
    const double *__restrict__ Za, const double *__restrict__ Wa, double *__restrict__ W, double *__restrict__ beta,
    double *__restrict__ V, double *__restrict__ Bst, float *__restrict__ d, const uint8_t *__restrict__ codes,
    const double *__restrict__ c, const int *__restrict__ active, const DevParams<double> &q, int64_t ldp,
    int store_b, double *__restrict__ gpart, const GateArgs &ga, NodeCols ncl, int64_t bx, int64_t by, int64_t gx,
    float *red) {
    constexpr int TM = 16 * BM, TN = 16 * BN, E = TM * TN / (64 * WAVES);
    static_assert(E * 64 * WAVES == TM * TN, "tile elements per thread");
    const int64_t m0 = bx * TM, n0 = by * TN;
    int sb[BN], se[E];
    if (!tile_slots<TM, BN, E, WAVES>(ncl, n0, sb, se)) return;
    EpiIn<double> ei[E];
    double za[E], wa[E];
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * WAVES;
        const int64_t col = n0 + idx / TM, j = m0 + idx % TM, o = col_row(se[t], col) * ldp + j;
        epi_load<double>(ei[t], se[t], col, j, ldp, W, V, codes, c, active);
        za[t] = Za[o];
        wa[t] = Wa[o];
    }
    nt_tile<float, float, float, BM, BN, WAVES>(A, lda, U, ldu, kdim, m0, n0, sb, red);
    const bool est = gpart != nullptr;
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * WAVES, n = idx / TM, m = idx % TM;
        double e[5] = {0, 0, 0, 0, 0};
        if (ei[t].on) {
            const int64_t o = (int64_t)se[t] * ldp + m0 + m;
            const double Qv = za[t] + (double)sum_waves<float, TM, TN, WAVES>(red, n, m);
            const double wn = admm_update<double>(Qv, ei[t], o, W, beta, V, Bst, q, store_b, est, ga, e);
            d[o] = (float)(wn - wa[t]);
        }
        if (est) store_estimate<TM>(e, m, se[t], gpart, gx, bx);
    }
}

template <int BM, int BN, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_admm_xtu_anch(
    const float *__restrict__ A, int64_t lda, const float *__restrict__ U, int64_t ldu, int64_t kdim,
    const double *__restrict__ Za, const double *__restrict__ Wa, double *__restrict__ W, double *__restrict__ beta,
    double *__restrict__ V, double *__restrict__ Bst, float *__restrict__ d, const uint8_t *__restrict__ codes,
    const double *__restrict__ c, const int *__restrict__ active, DevParams<double> q, int64_t ldp, int store_b,
    double *__restrict__ gpart, GateArgs ga, NodeCols ncl) {
    __shared__ float red[WAVES * Red<16 * BM, 16 * BN>::WS];
    xtu_anch_tile<BM, BN, WAVES>(A, lda, U, ldu, kdim, Za, Wa, W, beta, V, Bst, d, codes, c, active, q, ldp, store_b,
                                 gpart, ga, ncl, blockIdx.x, blockIdx.y, gridDim.x, red);
}

// ---------------------------------------------------------------------------
// Grouped launches (batching across instances).  One launch runs the same
// register-tile contraction (32 x 32 tile, 4 waves) for up to kGroupMax
// members, each with its own instance's operands, node batch and gx x gy tile
// grid: the launch's workgroups are the members' tiles one member after another
// (member g owns workgroups [tile0_g, tile0_g + gx_g gy_g), x fastest as in its
// own grid), so each tile computes exactly what the member's own launch would.
// ---------------------------------------------------------------------------
constexpr int kGroupMax = 8;

template <class T>
struct XwMember {
    const T *A, *B;
    T *U;
    const int *cols;
    int64_t lda, ldb, ldu, kdim;
    int gx, tile0;
};

template <class T>
struct XtuMember {
    const T *A, *U, *W, *c;
    T *Wout, *beta, *V, *Bst;
    const uint8_t *codes;
    const int *active, *cols;
    double *gpart;
    int64_t lda, ldu, kdim, ldp;
    int store_b, gx, tile0;
    DevParams<T> q;
    GateArgs ga;
};

struct AnchMember {
    const float *A, *U;
    const double *Za, *Wa, *c;
    double *W, *beta, *V, *Bst;
    float *d;
    const uint8_t *codes;
    const int *active, *cols;
    double *gpart;
    int64_t lda, ldu, kdim, ldp;
    int store_b, gx, tile0;
    DevParams<double> q;
    GateArgs ga;
};

template <class M>
struct Group {
    M m[kGroupMax];
    int count;
};

// Member owning workgroup b (members in tile order; uniform over the workgroup).
template <class M>
__device__ __forceinline__ int group_member(const Group<M> &g, int b) {
    int k = 0;
    for (int i = 1; i < g.count; ++i) k += b >= g.m[i].tile0;
    return k;
}

template <class T>
__global__ __launch_bounds__(256) void k_gemm_xw_grp(Group<XwMember<T>> g) {
    __shared__ T red[4 * Red<32, 32>::WS];
    const int b = blockIdx.x;
    const XwMember<T> &d = g.m[group_member(g, b)];
    const int loc = b - d.tile0;
    xw_tile<T, T, T, 2, 2, 4>(d.A, d.lda, d.B, d.ldb, d.U, d.ldu, d.kdim, NodeCols{d.cols}, 0, loc % d.gx,
                              loc / d.gx, 0, 1, red);
}

template <class T>
__global__ __launch_bounds__(256) void k_admm_xtu_grp(Group<XtuMember<T>> g) {
    __shared__ T red[4 * Red<32, 32>::WS];
    const int b = blockIdx.x;
    const XtuMember<T> &d = g.m[group_member(g, b)];
    const int loc = b - d.tile0;
    xtu_tile<T, T, 2, 2, 4>(d.A, d.lda, d.U, d.ldu, d.kdim, d.W, d.Wout, d.beta, d.V, d.Bst, d.codes, d.c, d.active,
                            d.q, d.ldp, d.store_b, d.gpart, d.ga, NodeCols{d.cols}, loc % d.gx, loc / d.gx, d.gx, red);
}

__global__ __launch_bounds__(256) void k_admm_xtu_anch_grp(Group<AnchMember> g) {
    __shared__ float red[4 * Red<32, 32>::WS];
    const int b = blockIdx.x;
    const AnchMember &d = g.m[group_member(g, b)];
    const int loc = b - d.tile0;
    xtu_anch_tile<2, 2, 4>(d.A, d.lda, d.U, d.ldu, d.kdim, d.Za, d.Wa, d.W, d.beta, d.V, d.Bst, d.d, d.codes, d.c,
                           d.active, d.q, d.ldp, d.store_b, d.gpart, d.ga, NodeCols{d.cols}, loc % d.gx, loc / d.gx,
                           d.gx, red);
}

static_assert(sizeof(Group<XtuMember<double>>) <= 4096 && sizeof(Group<AnchMember>) <= 4096,
              "a group travels in the kernel arguments");

// ---------------------------------------------------------------------------
// LDS-staged tiles for large grids.  A workgroup of 4 waves (2 x 2) owns a
// TM x TN output tile (TM = 32 WM, TN = 32 WN); every k chunk of 16 of the A
// slab (TM rows) and the B slab (TN node rows) is loaded once from global memory
// into LDS (two buffers: the next chunk's global loads are issued before the
// current chunk's MFMAs and stored after them) and each wave reads its
// (16 WM) x (16 WN) sub-tile's fragments from LDS, so a loaded element feeds
// 2 waves instead of 1 and the tile is 4-16 times larger than the register
// tiles' (far less L2 traffic per flop).  Each output element is owned by one
// lane (no cross-wave reduction).  Lane l reads 4 consecutive k of row l%16 for
// the 4 MFMAs of a chunk, as in nt_tile.  LDS rows hold 16 + pad elements
// (80 B for FP32, 144 B for FP64: 16 lanes' 16-byte reads spread over the banks).
// ---------------------------------------------------------------------------
template <class T> struct LdsRow;
template <> struct LdsRow<float> { static constexpr int LD = 20; };
template <> struct LdsRow<double> { static constexpr int LD = 18; };

template <class T, int WM, int WN>
struct LdsTile {
    static constexpr int TM = 32 * WM, TN = 32 * WN, LD = LdsRow<T>::LD;
    static constexpr int VPR = (int)sizeof(T);              // 16-byte vectors per 16-element row
    static constexpr int NA = TM * VPR / 256, NB = TN * VPR / 256;
    static constexpr int STAGE = (TM + TN) * LD;            // elements per buffer
};

template <class T, int WM, int WN>
__device__ __forceinline__ void lds_tile(const T *__restrict__ A, int64_t lda, const T *__restrict__ B, int64_t ldb,
                                         int64_t kdim, int64_t m0, int64_t n0, const NodeCols &ncl, T *smem,
                                         typename Acc<T>::type (&acc)[WM][WN]) {
    typedef LdsTile<T, WM, WN> L;
    constexpr int EPV = 16 / (int)sizeof(T);                 // elements per 16-byte vector
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int q = lane >> 4, r = lane & 15;
    typedef typename Acc<T>::type AccT;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = AccT{0, 0, 0, 0};
    // global source of each staged vector of this thread (row, 16-byte part)
    const T *ga[L::NA];
    const T *gb[L::NB];
    int la[L::NA], lb[L::NB];
#pragma unroll
    for (int e = 0; e < L::NA; ++e) {
        const int idx = tid + 256 * e, row = idx / L::VPR, part = idx % L::VPR;
        ga[e] = A + (m0 + row) * lda + EPV * part;
        la[e] = row * L::LD + EPV * part;
    }
#pragma unroll
    for (int e = 0; e < L::NB; ++e) {
        const int idx = tid + 256 * e, row = idx / L::VPR, part = idx % L::VPR;
        gb[e] = B + col_row(col_slot(ncl, n0 + row), n0 + row) * ldb + EPV * part;
        lb[e] = (L::TM + row) * L::LD + EPV * part;
    }
    float4 va[L::NA], vb[L::NB];
#define L0L2_GLOAD(c)                                                                                          \
    _Pragma("unroll") for (int e = 0; e < L::NA; ++e) va[e] = *reinterpret_cast<const float4 *>(ga[e] + 16 * (c)); \
    _Pragma("unroll") for (int e = 0; e < L::NB; ++e) vb[e] = *reinterpret_cast<const float4 *>(gb[e] + 16 * (c));
#define L0L2_SSTORE(st)                                                                                        \
    _Pragma("unroll") for (int e = 0; e < L::NA; ++e)                                                          \
        *reinterpret_cast<float4 *>(smem + (st) * L::STAGE + la[e]) = va[e];                                    \
    _Pragma("unroll") for (int e = 0; e < L::NB; ++e)                                                          \
        *reinterpret_cast<float4 *>(smem + (st) * L::STAGE + lb[e]) = vb[e];
    const int64_t nch = kdim / 16;
    L0L2_GLOAD(0)
    L0L2_SSTORE(0)
    __syncthreads();
    for (int64_t c = 0; c < nch; ++c) {
        const int st = (int)(c & 1);
        // next chunk (the last chunk reloads itself; its copy lands in the idle buffer)
        const int64_t cn = c + 1 < nch ? c + 1 : c;
        L0L2_GLOAD(cn)
        const T *sa = smem + st * L::STAGE;
        T a[WM][4], b[WN][4];
#pragma unroll
        for (int i = 0; i < WM; ++i) load4(sa + (wm * 16 * WM + 16 * i + r) * L::LD + 4 * q, a[i]);
#pragma unroll
        for (int j = 0; j < WN; ++j) load4(sa + (L::TM + wn * 16 * WN + 16 * j + r) * L::LD + 4 * q, b[j]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j) acc[i][j] = mfma16(a[i][t], b[j][t], acc[i][j]);
        L0L2_SSTORE(st ^ 1)
        __syncthreads();
    }
#undef L0L2_GLOAD
#undef L0L2_SSTORE
}

// Output position of accumulator v of block (i, j) held by this lane.
template <class T, int WM, int WN>
__device__ __forceinline__ void lds_pos(int i, int j, int v, int &m, int &n) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    m = (w >> 1) * 16 * WM + 16 * i + acc_row<T>(lane, v);
    n = (w & 1) * 16 * WN + 16 * j + (lane & 15);
}

// Epilogue of an LDS-staged tile.  A lane's accumulators cover 16 node columns
// and rows 4 apart, so writing node state straight from them scatters every
// access over 16 rows.  Instead the TM x TN tile goes to LDS node-major (row
// stride TM + 1: both the writes and the reads are free of bank conflicts) in
// NP passes of PN = TN / NP node columns (as many as the staging buffers hold),
// and each wave then takes whole node columns: lane l handles coordinates
// l + 64 h (h < TM / 64) of node column c0 + w + 4 t, so the node-state accesses
// of a wave are contiguous.
template <class TA, int WM, int WN>
struct LdsEpi {
    static constexpr int TM = 32 * WM, TN = 32 * WN, LD = TM + 1, H = TM / 64;
    // passes for a staging buffer of `bytes` bytes (0: not even a quarter fits)
    static constexpr int passes(size_t bytes) {
        return (size_t)TN * LD * sizeof(TA) <= bytes         ? 1
               : (size_t)(TN / 2) * LD * sizeof(TA) <= bytes ? 2
               : (size_t)(TN / 4) * LD * sizeof(TA) <= bytes ? 4
                                                               : 0;
    }
};

// Writes this lane's accumulators of node columns [c0, c0 + pn) to buf.
template <class TA, int WM, int WN>
__device__ __forceinline__ void acc_stage(const typename Acc<TA>::type (&acc)[WM][WN], TA *buf, int c0, int pn) {
    constexpr int LD = LdsEpi<TA, WM, WN>::LD;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            int m, n;
            lds_pos<TA, WM, WN>(i, j, 0, m, n);
            if (n < c0 || n >= c0 + pn) continue;   // whole 16-column block in or out
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                lds_pos<TA, WM, WN>(i, j, v, m, n);
                buf[(n - c0) * LD + m] = acc[i][j][v];
            }
        }
}

// Sum of each of the five estimate terms over the wave (every lane receives them).
__device__ __forceinline__ void wave_sum5(double e[5]) {
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int t = 0; t < 5; ++t) e[t] += __shfl_xor(e[t], off);
}

// Node-state operands of the coordinates m0 + lane + 64 h of one node column
// (col: its column index, slot: its list entry), all loaded before any update.
template <class T, int H>
__device__ __forceinline__ void epi_load_row(EpiIn<T> (&ei)[H], int slot, int64_t col, int64_t m0, int64_t ldp,
                                             const T *W, const T *__restrict__ V,
                                             const uint8_t *__restrict__ codes, const T *__restrict__ c,
                                             const int *__restrict__ active) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int h = 0; h < H; ++h) epi_load<T>(ei[h], slot, col, m0 + lane + 64 * h, ldp, W, V, codes, c, active);
}

// The node rows of a wave's epilogue pass, t = 0 .. T - 1 (T a multiple of D):
// the operands of rows t + 1 .. t + D - 1 are loaded (load(row, t')) before row
// t is updated (update(row, t)), so their latency overlaps D - 1 rows of work
// instead of being paid row by row.  The D rows sit in a ring of registers
// indexed with compile-time constants.
template <class Row, int D = 2, class Load, class Update>
__device__ __forceinline__ void rows_pipelined(int T, Load &&load, Update &&update) {
    Row ring[D];
    sfor<D - 1>([&](auto i) { load(ring[decltype(i)::value], decltype(i)::value); });
    for (int t = 0; t < T; t += D) {
        sfor<D>([&](auto i) {
            constexpr int k = decltype(i)::value, nxt = (k + D - 1) % D;
            if (t + k + D - 1 < T) load(ring[nxt], t + k + D - 1);
            update(ring[k], t + k);
        });
    }
}

// Contraction over p (U = Xh W^T) with an LDS-staged tile.  With gridDim.z = S
// > 1 the contraction range is cut into S equal slices (kdim / S a multiple of
// 16) and slice z writes its partial product to U + z pstride; k_splitk_sum adds
// the slices in order.  That gives a grid of S times as many workgroups when the
// output (n x nodes) is small and the range p long.
template <class T, int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm_xw_lds(const T *__restrict__ A, int64_t lda, const T *__restrict__ B,
                                                     int64_t ldb, T *__restrict__ U, int64_t ldu, int64_t kdim,
                                                     NodeCols ncl, int64_t pstride) {
    typedef LdsTile<T, WM, WN> L;
    __shared__ __align__(16) T smem[2 * L::STAGE];
    const int64_t m0 = (int64_t)blockIdx.x * L::TM, n0 = (int64_t)blockIdx.y * L::TN;
    if (col_slot(ncl, n0) < 0) return;
    const int64_t ks = kdim / gridDim.z, k0 = ks * blockIdx.z;
    U += pstride * blockIdx.z;
    typename Acc<T>::type acc[WM][WN];
    lds_tile<T, WM, WN>(A + k0, lda, B + k0, ldb, ks, m0, n0, ncl, smem, acc);
    typedef LdsEpi<T, WM, WN> E;
    constexpr int NP = E::passes(sizeof(smem));
    static_assert(NP > 0, "epilogue staging does not fit");
    constexpr int PN = L::TN / NP;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int pass = 0; pass < NP; ++pass) {
        const int c0 = pass * PN;
        __syncthreads();
        acc_stage<T, WM, WN>(acc, smem, c0, PN);
        __syncthreads();
        for (int t = 0; t < PN / 4; ++t) {
            const int nl = c0 + w + 4 * t, slot = col_slot(ncl, n0 + nl);
            if (slot < 0) continue;
#pragma unroll
            for (int h = 0; h < E::H; ++h)
                U[(int64_t)slot * ldu + m0 + lane + 64 * h] = smem[(nl - c0) * E::LD + lane + 64 * h];
        }
    }
}

// U[slot][m] = sum over the S slices of the partial products, in slice order,
// for the live columns.
template <class T>
__global__ __launch_bounds__(256) void k_splitk_sum(const T *__restrict__ P, int64_t pstride, int S,
                                                    T *__restrict__ U, int64_t ldu, int64_t rows, NodeCols ncl) {
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
    if (m >= rows) return;
    const int slot = col_slot(ncl, c);
    if (slot < 0) return;
    const int64_t o = (int64_t)slot * ldu + m;
    T v = P[o];
    for (int z = 1; z < S; ++z) v += P[z * pstride + o];
    U[o] = v;
}

// Contraction over n with the ADMM epilogue, LDS-staged tile.
template <class T, int WM, int WN>
__global__ __launch_bounds__(256) void k_admm_xtu_lds(const T *__restrict__ A, int64_t lda, const T *__restrict__ U,
                                                      int64_t ldu, int64_t kdim, const T *W, T *Wout,
                                                      T *__restrict__ beta, T *__restrict__ V, T *__restrict__ Bst,
                                                      const uint8_t *__restrict__ codes, const T *__restrict__ c,
                                                      const int *__restrict__ active, DevParams<T> q, int64_t ldp,
                                                      int store_b, double *__restrict__ gpart, GateArgs ga,
                                                      NodeCols ncl) {
    typedef LdsTile<T, WM, WN> L;
    __shared__ __align__(16) T smem[2 * L::STAGE];
    const int64_t m0 = (int64_t)blockIdx.x * L::TM, n0 = (int64_t)blockIdx.y * L::TN;
    if (col_slot(ncl, n0) < 0) return;
    typename Acc<T>::type acc[WM][WN];
    lds_tile<T, WM, WN>(A, lda, U, ldu, kdim, m0, n0, ncl, smem, acc);
    const bool est = gpart != nullptr;
    typedef LdsEpi<T, WM, WN> E;
    constexpr int NP = E::passes(sizeof(smem));
    static_assert(NP > 0, "epilogue staging does not fit");
    constexpr int PN = L::TN / NP;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int pass = 0; pass < NP; ++pass) {
        const int c0 = pass * PN;
        __syncthreads();
        acc_stage<T, WM, WN>(acc, smem, c0, PN);
        __syncthreads();
        for (int t = 0; t < PN / 4; ++t) {
            const int nl = c0 + w + 4 * t, slot = col_slot(ncl, n0 + nl);
            EpiIn<T> ei[E::H];
            epi_load_row<T, E::H>(ei, slot, n0 + nl, m0, ldp, W, V, codes, c, active);
            double e[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int h = 0; h < E::H; ++h) {
                if (!ei[h].on) continue;
                const int m = lane + 64 * h;
                double ev[5] = {0, 0, 0, 0, 0};
                admm_update<T>(smem[(nl - c0) * E::LD + m], ei[h], (int64_t)slot * ldp + m0 + m, Wout, beta, V, Bst,
                               q, store_b, est, ga, ev);
#pragma unroll
                for (int u = 0; u < 5; ++u) e[u] += ev[u];
            }
            if (est) {
                wave_sum5(e);
                if (lane == 0 && slot >= 0)
                    for (int u = 0; u < 5; ++u) gpart[((int64_t)slot * gridDim.x + blockIdx.x) * 5 + u] = e[u];
            }
        }
    }
}

// Contraction over n of an anchored sweep, LDS-staged tile.
template <int WM, int WN>
__global__ __launch_bounds__(256) void k_admm_xtu_anch_lds(
    const float *__restrict__ A, int64_t lda, const float *__restrict__ U, int64_t ldu, int64_t kdim,
    const double *__restrict__ Za, const double *__restrict__ Wa, double *__restrict__ W, double *__restrict__ beta,
    double *__restrict__ V, double *__restrict__ Bst, float *__restrict__ d, const uint8_t *__restrict__ codes,
    const double *__restrict__ c, const int *__restrict__ active, DevParams<double> q, int64_t ldp, int store_b,
    double *__restrict__ gpart, GateArgs ga, NodeCols ncl) {
    typedef LdsTile<float, WM, WN> L;
    __shared__ __align__(16) float smem[2 * L::STAGE];
    const int64_t m0 = (int64_t)blockIdx.x * L::TM, n0 = (int64_t)blockIdx.y * L::TN;
    if (col_slot(ncl, n0) < 0) return;
    f32x4 acc[WM][WN];
    lds_tile<float, WM, WN>(A, lda, U, ldu, kdim, m0, n0, ncl, smem, acc);
    const bool est = gpart != nullptr;
    typedef LdsEpi<float, WM, WN> E;
    constexpr int NP = E::passes(sizeof(smem));
    static_assert(NP > 0, "epilogue staging does not fit");
    constexpr int PN = L::TN / NP;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int pass = 0; pass < NP; ++pass) {
        const int c0 = pass * PN;
        __syncthreads();
        acc_stage<float, WM, WN>(acc, smem, c0, PN);
        __syncthreads();
        for (int t = 0; t < PN / 4; ++t) {
            const int nl = c0 + w + 4 * t, slot = col_slot(ncl, n0 + nl);
            EpiIn<double> ei[E::H];
            double za[E::H], wa[E::H];
            epi_load_row<double, E::H>(ei, slot, n0 + nl, m0, ldp, W, V, codes, c, active);
#pragma unroll
            for (int h = 0; h < E::H; ++h) {
                const int64_t o = col_row(slot, n0 + nl) * ldp + m0 + lane + 64 * h;
                za[h] = Za[o];
                wa[h] = Wa[o];
            }
            double e[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int h = 0; h < E::H; ++h) {
                if (!ei[h].on) continue;
                const int m = lane + 64 * h;
                const int64_t o = (int64_t)slot * ldp + m0 + m;
                double ev[5] = {0, 0, 0, 0, 0};
                const double wn = admm_update<double>(za[h] + (double)smem[(nl - c0) * E::LD + m], ei[h], o, W, beta,
                                                      V, Bst, q, store_b, est, ga, ev);
                d[o] = (float)(wn - wa[h]);
#pragma unroll
                for (int u = 0; u < 5; ++u) e[u] += ev[u];
            }
            if (est) {
                wave_sum5(e);
                if (lane == 0 && slot >= 0)
                    for (int u = 0; u < 5; ++u) gpart[((int64_t)slot * gridDim.x + blockIdx.x) * 5 + u] = e[u];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// BF16 form of the two contractions: the folded operand is stored as two BF16
// terms (hi + lo), the FP32 node operand is split into two BF16 terms on load,
// and each 16 x 16 block accumulates hi*hi + hi*lo + lo*hi in FP32 (the lo*lo
// term is below FP32 resolution).  Lane l supplies 8 consecutive k of row l%16
// (16x16x32 MFMA); the contraction over p reads the row-major copy, the
// contraction over n the column-major copy.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void split8(const float w[8], bf16x8 &hi, bf16x8 &lo) {
    for (int t = 0; t < 8; ++t) {
        __bf16 h = (__bf16)w[t];
        hi[t] = h;
        lo[t] = (__bf16)(w[t] - (float)h);
    }
}

// The same split of four values (a staged 16-byte vector).
__device__ __forceinline__ void split4(const float4 &w, bf16x4 &hi, bf16x4 &lo) {
    const float x[4] = {w.x, w.y, w.z, w.w};
    for (int t = 0; t < 4; ++t) {
        __bf16 h = (__bf16)x[t];
        hi[t] = h;
        lo[t] = (__bf16)(x[t] - (float)h);
    }
}

__device__ __forceinline__ void split4(const f32x4 &w, bf16x4 &hi, bf16x4 &lo) {
    for (int t = 0; t < 4; ++t) {
        __bf16 h = (__bf16)w[t];
        hi[t] = h;
        lo[t] = (__bf16)(w[t] - (float)h);
    }
}

__device__ __forceinline__ void load8f(const float *p, float out[8]) {
    float4 a = *reinterpret_cast<const float4 *>(p);
    float4 b = *reinterpret_cast<const float4 *>(p + 4);
    out[0] = a.x; out[1] = a.y; out[2] = a.z; out[3] = a.w;
    out[4] = b.x; out[5] = b.y; out[6] = b.z; out[7] = b.w;
}

// 32 x 32 tile of C[m][n] = sum_k (Ahi + Alo)[m][k] B[n][k] with A rows in BF16
// (hi, lo) and B rows in FP32 (split into hi, lo on load); chunks of 32 k split
// in pairs over WAVES waves, next chunk's loads issued before the current
// chunk's MFMAs with the branch-free loop of nt_tile.  kdim must be a multiple
// of 64.
template <int WAVES>
__device__ __forceinline__ void nt_tile_bf16(const __bf16 *__restrict__ Ahi, const __bf16 *__restrict__ Alo,
                                             int64_t lda, const float *__restrict__ B, int64_t ldb, int64_t kdim,
                                             int64_t m0, int64_t n0, const int (&sb)[2], float *red,
                                             int64_t pr0 = 0, int64_t pr1 = -1) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int q = lane >> 4, r = lane & 15;
    const int64_t brow[2] = {col_row(sb[0], n0 + r), col_row(sb[1], n0 + 16 + r)};
    f32x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0, 0, 0, 0};
    // pairs [pr0, pr1) of 64 k (all of kdim by default), split over the waves
    if (pr1 < 0) pr1 = kdim / 64;
    const int64_t npr = pr1 - pr0;
    const int wu = __builtin_amdgcn_readfirstlane(w);
    const int64_t c0 = 2 * (pr0 + npr * wu / WAVES), c1 = 2 * (pr0 + npr * (wu + 1) / WAVES);
    bf16x8 ah[2][2], al[2][2];
    float bv[2][2][8];
    auto load = [&](int st, int64_t c) {
        for (int a = 0; a < 2; ++a) {
            const int64_t o = (m0 + 16 * a + r) * lda + 32 * c + 8 * q;
            ah[st][a] = *reinterpret_cast<const bf16x8 *>(Ahi + o);
            al[st][a] = *reinterpret_cast<const bf16x8 *>(Alo + o);
        }
        for (int b = 0; b < 2; ++b) load8f(B + brow[b] * ldb + 32 * c + 8 * q, bv[st][b]);
        __builtin_amdgcn_sched_barrier(0);
    };
    auto compute = [&](int st) {
        bf16x8 bh[2], bl[2];
        for (int b = 0; b < 2; ++b) split8(bv[st][b], bh[b], bl[b]);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                acc[a][b] = mfma16_bf16(ah[st][a], bh[b], acc[a][b]);
                acc[a][b] = mfma16_bf16(ah[st][a], bl[b], acc[a][b]);
                acc[a][b] = mfma16_bf16(al[st][a], bh[b], acc[a][b]);
            }
    };
    if (c0 < c1) {
        load(0, c0);
        int64_t c = c0;
        for (; c + 2 < c1; c += 2) {
            load(1, c + 1);
            compute(0);
            __builtin_amdgcn_sched_barrier(0);
            load(0, c + 2);
            compute(1);
            __builtin_amdgcn_sched_barrier(0);
        }
        load(1, c + 1);
        compute(0);
        compute(1);
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int v = 0; v < 4; ++v) {
                int m = a * 16 + acc_row<float>(lane, v);
                int n = b * 16 + r;
                red[w * Red<32, 32>::WS + n * Red<32, 32>::LD + m] = acc[a][b][v];
            }
    __syncthreads();
}

// LDS-staged tile of the BF16 split form (4 waves, 2 x 2; TM = 32 WM, TN = 32 WN).
// A k chunk of 32 stages, per row, the BF16 hi and lo terms (2 x 64 B) of A and
// of B (whose FP32 values are split as they are staged), each row padded to
// 144 B; lane l reads 8 consecutive k of row l%16, one 16-byte read per term.
template <int WM, int WN>
struct LdsTileBf {
    static constexpr int TM = 32 * WM, TN = 32 * WN;
    static constexpr int ROWB = 144;                         // bytes per staged row
    static constexpr int NA = TM * 8 / 256, NB = TN * 8 / 256;   // 16-byte vectors per thread
    static constexpr int STAGE = (TM + TN) * ROWB;           // bytes per buffer
};

template <int WM, int WN>
__device__ __forceinline__ void lds_tile_bf16(const __bf16 *__restrict__ Ahi, const __bf16 *__restrict__ Alo,
                                              int64_t lda, const float *__restrict__ B, int64_t ldb, int64_t kdim,
                                              int64_t m0, int64_t n0, const NodeCols &ncl,
                                              unsigned char *smem, f32x4 (&acc)[WM][WN]) {
    typedef LdsTileBf<WM, WN> L;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int q = lane >> 4, r = lane & 15;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    // staged vector e of this thread: row idx / 8, part idx % 8 (A: parts 0-3 hi,
    // 4-7 lo; B: parts 0-7 of the FP32 row, each 4 values split into BF16 hi and
    // lo as they are staged, so a B row in LDS has the layout of an A row: 32 hi
    // terms, then 32 lo terms, and every element is split once per workgroup
    // rather than once per wave that reads it)
    const unsigned char *ga[L::NA];
    const unsigned char *gb[L::NB];
    int la[L::NA], lb[L::NB];
#pragma unroll
    for (int e = 0; e < L::NA; ++e) {
        const int idx = tid + 256 * e, row = idx >> 3, part = idx & 7;
        const __bf16 *src = (part < 4 ? Ahi : Alo) + (m0 + row) * lda;
        ga[e] = reinterpret_cast<const unsigned char *>(src) + 16 * (part & 3);
        la[e] = row * L::ROWB + 16 * part;
    }
#pragma unroll
    for (int e = 0; e < L::NB; ++e) {
        const int idx = tid + 256 * e, row = idx >> 3, part = idx & 7;
        gb[e] = reinterpret_cast<const unsigned char *>(B + col_row(col_slot(ncl, n0 + row), n0 + row) * ldb) +
                16 * part;
        lb[e] = (L::TM + row) * L::ROWB + 8 * part;
    }
    // two register sets: chunk c + 2's loads are issued while chunk c is
    // multiplied, chunk c + 1's (issued a chunk earlier) are staged after it;
    // the arrays are indexed with compile-time constants (sfor) only
    f32x4 va0[L::NA], vb0[L::NB], va1[L::NA], vb1[L::NB];
    // chunk c covers 32 k: 64 bytes of each BF16 term, 128 bytes of FP32
#define L0L2_GLOADB(VA, VB, c)                                                                              \
    {                                                                                                       \
        const int64_t c_ = (c);                                                                             \
        sfor<L::NA>([&](auto e) { VA[e] = *reinterpret_cast<const f32x4 *>(ga[e] + 64 * c_); });           \
        sfor<L::NB>([&](auto e) { VB[e] = *reinterpret_cast<const f32x4 *>(gb[e] + 128 * c_); });          \
    }                                                                                                       \
    __builtin_amdgcn_sched_barrier(0);
#define L0L2_SSTOREB(st, VA, VB)                                                                            \
    sfor<L::NA>([&](auto e) { *reinterpret_cast<f32x4 *>(smem + (st) * L::STAGE + la[e]) = VA[e]; });      \
    sfor<L::NB>([&](auto e) {                                                                               \
        bf16x4 h4, l4;                                                                                      \
        split4(VB[e], h4, l4);                                                                              \
        *reinterpret_cast<bf16x4 *>(smem + (st) * L::STAGE + lb[e]) = h4;                                    \
        *reinterpret_cast<bf16x4 *>(smem + (st) * L::STAGE + lb[e] + 64) = l4;                               \
    });
#define L0L2_COMPUTEB(st)                                                                                   \
    {                                                                                                       \
        const unsigned char *sa = smem + (st) * L::STAGE;                                                   \
        bf16x8 bh[WN], bl[WN];                                                                              \
        _Pragma("unroll") for (int j = 0; j < WN; ++j) {                                                    \
            const unsigned char *row = sa + (L::TM + wn * 16 * WN + 16 * j + r) * L::ROWB;                  \
            bh[j] = *reinterpret_cast<const bf16x8 *>(row + 16 * q);                                        \
            bl[j] = *reinterpret_cast<const bf16x8 *>(row + 64 + 16 * q);                                   \
        }                                                                                                   \
        _Pragma("unroll") for (int i = 0; i < WM; ++i) {                                                    \
            const unsigned char *row = sa + (wm * 16 * WM + 16 * i + r) * L::ROWB;                          \
            const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(row + 16 * q);                              \
            const bf16x8 al = *reinterpret_cast<const bf16x8 *>(row + 64 + 16 * q);                         \
            _Pragma("unroll") for (int j = 0; j < WN; ++j) {                                                \
                acc[i][j] = mfma16_bf16(ah, bh[j], acc[i][j]);                                              \
                acc[i][j] = mfma16_bf16(ah, bl[j], acc[i][j]);                                              \
                acc[i][j] = mfma16_bf16(al, bh[j], acc[i][j]);                                              \
            }                                                                                               \
        }                                                                                                   \
    }
    // chunks past the last re-load the last one (in bounds, never staged)
    const int64_t nch = kdim / 32, last = nch - 1;
    L0L2_GLOADB(va0, vb0, 0)
    L0L2_GLOADB(va1, vb1, last < 1 ? last : 1)
    L0L2_SSTOREB(0, va0, vb0)
    __syncthreads();
    // pairs of chunks with no branch inside the body: a branch between a load
    // and its use lets the compiler sink the load past it, which cuts that
    // load's head start from two chunks of work to one
    int64_t c = 0;
    for (; c + 1 < nch; c += 2) {
        L0L2_GLOADB(va0, vb0, c + 2 < last ? c + 2 : last)
        L0L2_COMPUTEB(0)
        __builtin_amdgcn_sched_barrier(0);
        L0L2_SSTOREB(1, va1, vb1)
        __syncthreads();
        L0L2_GLOADB(va1, vb1, c + 3 < last ? c + 3 : last)
        L0L2_COMPUTEB(1)
        __builtin_amdgcn_sched_barrier(0);
        L0L2_SSTOREB(0, va0, vb0)
        __syncthreads();
    }
    if (c < nch) {
        // odd count: the last chunk is in stage 0
        L0L2_COMPUTEB(0)
    }
#undef L0L2_GLOADB
#undef L0L2_SSTOREB
#undef L0L2_COMPUTEB
}

// BF16 split form, contraction over p, LDS-staged tile.  With gridDim.z = S > 1,
// slice z takes the chunks [nch z / S, nch (z + 1) / S) of 32 k (the launcher
// keeps S <= nch) and writes its partial product to U + z pstride.
template <int WM, int WN>
__global__ __launch_bounds__(256, 2) void k_gemm_xw_bf16_lds(const __bf16 *__restrict__ Ahi,
                                                          const __bf16 *__restrict__ Alo, int64_t lda,
                                                          const float *__restrict__ B, int64_t ldb,
                                                          float *__restrict__ U, int64_t ldu, int64_t kdim,
                                                          NodeCols ncl, int64_t pstride) {
    typedef LdsTileBf<WM, WN> L;
    __shared__ __align__(16) unsigned char smem[2 * L::STAGE];
    const int64_t m0 = (int64_t)blockIdx.x * L::TM, n0 = (int64_t)blockIdx.y * L::TN;
    if (col_slot(ncl, n0) < 0) return;
    const int64_t nch = kdim / 32, z = blockIdx.z, S = gridDim.z;
    const int64_t c0 = nch * z / S, c1 = nch * (z + 1) / S;
    U += pstride * z;
    f32x4 acc[WM][WN];
    lds_tile_bf16<WM, WN>(Ahi + 32 * c0, Alo + 32 * c0, lda, B + 32 * c0, ldb, 32 * (c1 - c0), m0, n0, ncl, smem,
                          acc);
    typedef LdsEpi<float, WM, WN> E;
    constexpr int NP = E::passes(sizeof(smem));
    static_assert(NP > 0, "epilogue staging does not fit");
    constexpr int PN = L::TN / NP;
    float *buf = reinterpret_cast<float *>(smem);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int pass = 0; pass < NP; ++pass) {
        const int c0 = pass * PN;
        __syncthreads();
        acc_stage<float, WM, WN>(acc, buf, c0, PN);
        __syncthreads();
        for (int t = 0; t < PN / 4; ++t) {
            const int nl = c0 + w + 4 * t, slot = col_slot(ncl, n0 + nl);
            if (slot < 0) continue;
#pragma unroll
            for (int h = 0; h < E::H; ++h)
                U[(int64_t)slot * ldu + m0 + lane + 64 * h] = buf[(nl - c0) * E::LD + lane + 64 * h];
        }
    }
}

// BF16 split form, contraction over n with the FP32 ADMM epilogue (anch == 0)
// or the anchored FP64 epilogue (anch == 1: Q = z_a + Q_bf16, FP64 state,
// d = fl32(W - w_a) into dst32), LDS-staged tile.  anch == 2: the first sweep
// of a block of single-term sweeps (Gram form, FP32 state): the FP32 update as
// for anch == 0, and this sweep's product and operand become the block's FP32
// anchor (Za32 = G w, Wa32 = w) with the next operand d = bf16(W_new - w) in Dout.
template <int WM, int WN, int ANCH>
__global__ __launch_bounds__(256, 2) void k_admm_xtu_bf16_lds(
    const __bf16 *__restrict__ Ahi, const __bf16 *__restrict__ Alo, int64_t lda, const float *__restrict__ U,
    int64_t ldu, int64_t kdim, const float *W32, float *W32out, float *__restrict__ beta32, float *__restrict__ V32,
    float *__restrict__ B32, const double *__restrict__ Za, const double *__restrict__ Wa, double *__restrict__ W64,
    double *__restrict__ beta64, double *__restrict__ V64, double *__restrict__ B64, const uint8_t *__restrict__ codes,
    const float *__restrict__ c32, const double *__restrict__ c64, const int *__restrict__ active,
    DevParams<float> q32, DevParams<double> q64, int64_t ldp, int store_b, double *__restrict__ gpart, GateArgs ga,
    NodeCols ncl, float *__restrict__ Za32 = nullptr, float *__restrict__ Wa32 = nullptr,
    __bf16 *__restrict__ Dout = nullptr) {
    typedef LdsTileBf<WM, WN> L;
    __shared__ __align__(16) unsigned char smem[2 * L::STAGE];
    const int64_t m0 = (int64_t)blockIdx.x * L::TM, n0 = (int64_t)blockIdx.y * L::TN;
    if (col_slot(ncl, n0) < 0) return;
    f32x4 acc[WM][WN];
    lds_tile_bf16<WM, WN>(Ahi, Alo, lda, U, ldu, kdim, m0, n0, ncl, smem, acc);
    const bool est = gpart != nullptr;
    typedef LdsEpi<float, WM, WN> E;
    constexpr int NP = E::passes(sizeof(smem));
    static_assert(NP > 0, "epilogue staging does not fit");
    constexpr int PN = L::TN / NP;
    float *buf = reinterpret_cast<float *>(smem);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int pass = 0; pass < NP; ++pass) {
        const int c0 = pass * PN;
        __syncthreads();
        acc_stage<float, WM, WN>(acc, buf, c0, PN);
        __syncthreads();
        typedef typename std::conditional<ANCH == 1, double, float>::type ST;
        struct Row {
            EpiIn<ST> ei[E::H];
            double za[ANCH == 1 ? E::H : 1], wa[ANCH == 1 ? E::H : 1];
            int slot;
        };
        auto load = [&](Row &R, int t) {
            const int nl = c0 + w + 4 * t;
            R.slot = col_slot(ncl, n0 + nl);
            if constexpr (ANCH == 1) {
                epi_load_row<double, E::H>(R.ei, R.slot, n0 + nl, m0, ldp, W64, V64, codes, c64, active);
#pragma unroll
                for (int h = 0; h < E::H; ++h) {
                    const int64_t o = col_row(R.slot, n0 + nl) * ldp + m0 + lane + 64 * h;
                    R.za[h] = Za[o];
                    R.wa[h] = Wa[o];
                }
            } else {
                epi_load_row<float, E::H>(R.ei, R.slot, n0 + nl, m0, ldp, W32, V32, codes, c32, active);
            }
        };
        auto update = [&](const Row &R, int t) {
            const int nl = c0 + w + 4 * t, slot = R.slot;
            double e[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int h = 0; h < E::H; ++h) {
                if (!R.ei[h].on) continue;
                const int m = lane + 64 * h;
                const int64_t o = (int64_t)slot * ldp + m0 + m;
                double ev[5] = {0, 0, 0, 0, 0};
                if constexpr (ANCH == 1) {
                    const double wn = admm_update<double>(R.za[h] + (double)buf[(nl - c0) * E::LD + m], R.ei[h], o,
                                                          W64, beta64, V64, B64, q64, store_b, est, ga, ev);
                    W32out[o] = (float)(wn - R.wa[h]);
                } else {
                    const float qv = buf[(nl - c0) * E::LD + m];
                    const float wn = admm_update<float>(qv, R.ei[h], o, W32out, beta32, V32, B32, q32, store_b, est,
                                                        ga, ev);
                    if (ANCH == 2) {
                        Za32[o] = qv;
                        Wa32[o] = R.ei[h].w;
                        Dout[o] = (__bf16)(wn - R.ei[h].w);
                    }
                }
#pragma unroll
                for (int u = 0; u < 5; ++u) e[u] += ev[u];
            }
            if (est) {
                wave_sum5(e);
                if (lane == 0 && slot >= 0)
                    for (int u = 0; u < 5; ++u) gpart[((int64_t)slot * gridDim.x + blockIdx.x) * 5 + u] = e[u];
            }
        };
        static_assert((PN / 4) % 2 == 0, "rows per wave in pairs");
        rows_pipelined<Row>(PN / 4, load, update);
    }
}

// LDS-staged tile of the single-term BF16 form: A and B are BF16 arrays (one
// term each); a k chunk of 64 stages the 128 bytes of each row (padded to 144 B,
// the split form's geometry), and each 16x16x32 MFMA pair covers the chunk's two
// 32-wide halves (lane l reads 8 consecutive k of row l % 16 in each half).  One
// MFMA per 32 k of the product, a third of the split form's three.
template <int WM, int WN>
__device__ __forceinline__ void lds_tile_bf16s(const __bf16 *__restrict__ A, int64_t lda,
                                               const __bf16 *__restrict__ B, int64_t ldb, int64_t kdim, int64_t m0,
                                               int64_t n0, const NodeCols &ncl, unsigned char *smem,
                                               f32x4 (&acc)[WM][WN]) {
    typedef LdsTileBf<WM, WN> L;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int q = lane >> 4, r = lane & 15;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    // staged vector e of this thread: row idx / 8, bytes 16 (idx % 8) .. + 15 of the row's chunk
    const unsigned char *ga[L::NA];
    const unsigned char *gb[L::NB];
    int la[L::NA], lb[L::NB];
#pragma unroll
    for (int e = 0; e < L::NA; ++e) {
        const int idx = tid + 256 * e, row = idx >> 3, part = idx & 7;
        ga[e] = reinterpret_cast<const unsigned char *>(A + (m0 + row) * lda) + 16 * part;
        la[e] = row * L::ROWB + 16 * part;
    }
#pragma unroll
    for (int e = 0; e < L::NB; ++e) {
        const int idx = tid + 256 * e, row = idx >> 3, part = idx & 7;
        gb[e] = reinterpret_cast<const unsigned char *>(B + col_row(col_slot(ncl, n0 + row), n0 + row) * ldb) +
                16 * part;
        lb[e] = (L::TM + row) * L::ROWB + 16 * part;
    }
    // two register sets of staged vectors: the loads of chunk c + 2 are issued
    // while chunk c is multiplied, and those of chunk c + 1 (a whole chunk
    // earlier) are stored to the other LDS stage after it, so each chunk's loads
    // have two chunks of MFMA work to arrive
    f32x4 va0[L::NA], vb0[L::NB], va1[L::NA], vb1[L::NB];
    // the staging loops index their arrays with compile-time constants (sfor),
    // so the register sets never become stack arrays
#define L0L2_GLOADS(VA, VB, c)                                                                              \
    {                                                                                                       \
        const int64_t off_ = 128 * (c);                                                                     \
        sfor<L::NA>([&](auto e) { VA[e] = *reinterpret_cast<const f32x4 *>(ga[e] + off_); });             \
        sfor<L::NB>([&](auto e) { VB[e] = *reinterpret_cast<const f32x4 *>(gb[e] + off_); });             \
    }                                                                                                       \
    __builtin_amdgcn_sched_barrier(0);
#define L0L2_SSTORES(st, VA, VB)                                                                            \
    sfor<L::NA>([&](auto e) { *reinterpret_cast<f32x4 *>(smem + (st) * L::STAGE + la[e]) = VA[e]; });     \
    sfor<L::NB>([&](auto e) { *reinterpret_cast<f32x4 *>(smem + (st) * L::STAGE + lb[e]) = VB[e]; });
#define L0L2_COMPUTES(st)                                                                                   \
    {                                                                                                       \
        const unsigned char *sa = smem + (st) * L::STAGE;                                                   \
        bf16x8 b0[WN], b1[WN];                                                                              \
        _Pragma("unroll") for (int j = 0; j < WN; ++j) {                                                    \
            const unsigned char *row = sa + (L::TM + wn * 16 * WN + 16 * j + r) * L::ROWB;                  \
            b0[j] = *reinterpret_cast<const bf16x8 *>(row + 16 * q);                                        \
            b1[j] = *reinterpret_cast<const bf16x8 *>(row + 64 + 16 * q);                                   \
        }                                                                                                   \
        _Pragma("unroll") for (int i = 0; i < WM; ++i) {                                                    \
            const unsigned char *row = sa + (wm * 16 * WM + 16 * i + r) * L::ROWB;                          \
            const bf16x8 a0 = *reinterpret_cast<const bf16x8 *>(row + 16 * q);                              \
            const bf16x8 a1 = *reinterpret_cast<const bf16x8 *>(row + 64 + 16 * q);                         \
            _Pragma("unroll") for (int j = 0; j < WN; ++j) {                                                \
                acc[i][j] = mfma16_bf16(a0, b0[j], acc[i][j]);                                              \
                acc[i][j] = mfma16_bf16(a1, b1[j], acc[i][j]);                                              \
            }                                                                                               \
        }                                                                                                   \
    }
    // chunks past the last re-load the last one (in bounds, never stored)
    const int64_t nch = kdim / 64, last = nch - 1;
    L0L2_GLOADS(va0, vb0, 0)
    L0L2_GLOADS(va1, vb1, last < 1 ? last : 1)
    L0L2_SSTORES(0, va0, vb0)
    __syncthreads();
    // pairs of chunks with no branch inside the body (a branch between a load
    // and its use lets the compiler sink the load past it, which cuts that
    // load's head start from two chunks of work to one)
    int64_t c = 0;
    for (; c + 1 < nch; c += 2) {
        // chunk c in LDS stage 0, chunk c + 1 in register set 1
        L0L2_GLOADS(va0, vb0, c + 2 < last ? c + 2 : last)
        L0L2_COMPUTES(0)
        __builtin_amdgcn_sched_barrier(0);
        L0L2_SSTORES(1, va1, vb1)
        __syncthreads();
        // chunk c + 1 in LDS stage 1, chunk c + 2 in register set 0
        L0L2_GLOADS(va1, vb1, c + 3 < last ? c + 3 : last)
        L0L2_COMPUTES(1)
        __builtin_amdgcn_sched_barrier(0);
        L0L2_SSTORES(0, va0, vb0)
        __syncthreads();
    }
    if (c < nch) {
        // odd count: the last chunk is in stage 0
        L0L2_COMPUTES(0)
    }
#undef L0L2_GLOADS
#undef L0L2_SSTORES
#undef L0L2_COMPUTES
}

// Anchored single-term sweep of the Gram form: Q = z + G_bf16 d_bf16, where d is
// the movement since the block's anchor (w = w_a + d) and z = G w_a.  MODE 1: FP32
// state with the FP32 anchor (Za32, Wa32) of the block's first sweep; MODE 2:
// FP64 state with the FP64 anchor (Za, Wa).  Both write the next operand
// d = bf16(W_new - w_a) to Dout.  The product's rounding error scales with |d|,
// which vanishes as the iterates settle, so the single BF16 term costs the
// fixed point nothing that the anchor does not already fix.
// The 256-row tile (WM = 8) keeps one workgroup per compute unit (its LDS
// stages and accumulators need the whole budget) and reports the gap-estimate
// sums per 128-row half, the granularity the 128-row tiles report.
template <int WM, int WN, int MODE>
__global__ __launch_bounds__(256, (WM > 4 ? 1 : 2)) void k_admm_xtu_bf16s_lds(
    const __bf16 *__restrict__ A, int64_t lda, const __bf16 *__restrict__ Din, __bf16 *__restrict__ Dout,
    int64_t kdim, const float *W32, float *W32out, float *__restrict__ beta32, float *__restrict__ V32,
    float *__restrict__ B32, const float *__restrict__ Za32, const float *__restrict__ Wa32,
    const double *__restrict__ Za, const double *__restrict__ Wa, double *__restrict__ W64,
    double *__restrict__ beta64, double *__restrict__ V64, double *__restrict__ B64, const uint8_t *__restrict__ codes,
    const float *__restrict__ c32, const double *__restrict__ c64, const int *__restrict__ active,
    DevParams<float> q32, DevParams<double> q64, int64_t ldp, int store_b, double *__restrict__ gpart, GateArgs ga,
    NodeCols ncl) {
    typedef LdsTileBf<WM, WN> L;
    __shared__ __align__(16) unsigned char smem[2 * L::STAGE];
    const int64_t m0 = (int64_t)blockIdx.x * L::TM, n0 = (int64_t)blockIdx.y * L::TN;
    if (col_slot(ncl, n0) < 0) return;
    f32x4 acc[WM][WN];
    lds_tile_bf16s<WM, WN>(A, lda, Din, ldp, kdim, m0, n0, ncl, smem, acc);
    const bool est = gpart != nullptr;
    typedef LdsEpi<float, WM, WN> E;
    constexpr int NP = E::passes(sizeof(smem));
    static_assert(NP > 0, "epilogue staging does not fit");
    constexpr int PN = L::TN / NP;
    float *buf = reinterpret_cast<float *>(smem);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // estimate sums per 128-row part of the tile (one part for tiles up to 128 rows)
    constexpr int NH = L::TM > 128 ? L::TM / 128 : 1, HP = E::H / NH;
    const int64_t ntile = (int64_t)gridDim.x * NH;
    for (int pass = 0; pass < NP; ++pass) {
        const int c0 = pass * PN;
        __syncthreads();
        acc_stage<float, WM, WN>(acc, buf, c0, PN);
        __syncthreads();
        typedef typename std::conditional<MODE == 2, double, float>::type ST;
        struct Row {
            EpiIn<ST> ei[E::H];
            ST za[E::H], wa[E::H];
            int slot;
        };
        auto load_row = [&](Row &R, int t) {
            const int nl = c0 + w + 4 * t;
            R.slot = col_slot(ncl, n0 + nl);
            if constexpr (MODE == 2)
                epi_load_row<double, E::H>(R.ei, R.slot, n0 + nl, m0, ldp, W64, V64, codes, c64, active);
            else
                epi_load_row<float, E::H>(R.ei, R.slot, n0 + nl, m0, ldp, W32, V32, codes, c32, active);
#pragma unroll
            for (int h = 0; h < E::H; ++h) {
                const int64_t o = col_row(R.slot, n0 + nl) * ldp + m0 + lane + 64 * h;
                if constexpr (MODE == 2) {
                    R.za[h] = Za[o];
                    R.wa[h] = Wa[o];
                } else {
                    R.za[h] = Za32[o];
                    R.wa[h] = Wa32[o];
                }
            }
        };
        auto update_row = [&](const Row &R, int t) {
            const int nl = c0 + w + 4 * t, slot = R.slot;
            double e[NH][5] = {};
#pragma unroll
            for (int h = 0; h < E::H; ++h) {
                if (!R.ei[h].on) continue;
                const int m = lane + 64 * h;
                const int64_t o = (int64_t)slot * ldp + m0 + m;
                double ev[5] = {0, 0, 0, 0, 0};
                if constexpr (MODE == 2) {
                    const double wn = admm_update<double>(R.za[h] + (double)buf[(nl - c0) * E::LD + m], R.ei[h], o,
                                                          W64, beta64, V64, B64, q64, store_b, est, ga, ev);
                    Dout[o] = (__bf16)(float)(wn - R.wa[h]);
                } else {
                    const float wn = admm_update<float>(R.za[h] + buf[(nl - c0) * E::LD + m], R.ei[h], o, W32out,
                                                        beta32, V32, B32, q32, store_b, est, ga, ev);
                    Dout[o] = (__bf16)(wn - R.wa[h]);
                }
#pragma unroll
                for (int u = 0; u < 5; ++u) e[h / HP][u] += ev[u];
            }
            if (est) {
#pragma unroll
                for (int hh = 0; hh < NH; ++hh) {
                    wave_sum5(e[hh]);
                    if (lane == 0 && slot >= 0)
                        for (int u = 0; u < 5; ++u)
                            gpart[((int64_t)slot * ntile + (int64_t)blockIdx.x * NH + hh) * 5 + u] = e[hh][u];
                }
            }
        };
        static_assert((PN / 4) % 4 == 0, "rows per wave in fours");
        rows_pipelined<Row, 4>(PN / 4, load_row, update_row);
    }
}

// Start of an anchored single-term block (FP64 state): w_a = W (FP64) and the
// operand of the block's first sweep d = 0.
__global__ void k_anchor_init_bf(const double *__restrict__ W, double *__restrict__ Wa, __bf16 *__restrict__ d,
                                 int64_t total) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        Wa[idx] = W[idx];
        d[idx] = (__bf16)0.0f;
    }
}

constexpr int kWavesBf16 = 8;

// U[k][i] = sum_j Xh[i][j] W[k][j] with Xh row-major (row i at A + i*lda); with
// gridDim.z = S > 1, slices of the range write partial products to U + z pstride
// as in k_gemm_xw.
__device__ __forceinline__ void xw_bf16_tile(const __bf16 *__restrict__ Ahi, const __bf16 *__restrict__ Alo,
                                             int64_t lda, const float *__restrict__ B, int64_t ldb,
                                             float *__restrict__ U, int64_t ldu, int64_t kdim, NodeCols ncl,
                                             int64_t pstride, int64_t bx, int64_t by, int64_t z, int64_t S,
                                             float *red) {
    const int64_t m0 = bx * 32, n0 = by * 32;
    constexpr int E = 1024 / (64 * kWavesBf16);
    int sb[2], se[E];
    if (!tile_slots<32, 2, E, kWavesBf16>(ncl, n0, sb, se)) return;
    const int64_t npr = kdim / 64;
    U += pstride * z;
    nt_tile_bf16<kWavesBf16>(Ahi, Alo, lda, B, ldb, kdim, m0, n0, sb, red, npr * z / S, npr * (z + 1) / S);
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * kWavesBf16, n = idx >> 5, m = idx & 31;
        if (se[t] >= 0) U[(int64_t)se[t] * ldu + m0 + m] = sum_waves<float, 32, 32, kWavesBf16>(red, n, m);
    }
}

__global__ __launch_bounds__(64 * kWavesBf16) void k_gemm_xw_bf16(const __bf16 *__restrict__ Ahi,
                                                                  const __bf16 *__restrict__ Alo, int64_t lda,
                                                                  const float *__restrict__ B, int64_t ldb,
                                                                  float *__restrict__ U, int64_t ldu, int64_t kdim,
                                                                  NodeCols ncl, int64_t pstride) {
    __shared__ float red[kWavesBf16 * Red<32, 32>::WS];
    xw_bf16_tile(Ahi, Alo, lda, B, ldb, U, ldu, kdim, ncl, pstride, blockIdx.x, blockIdx.y, blockIdx.z, gridDim.z,
                 red);
}

// Q[k][j] = sum_i Xh[i][j] U[k][i] (Xh column-major) with the ADMM epilogue.
__device__ __forceinline__ void xtu_bf16_tile(
    const __bf16 *__restrict__ Ahi, const __bf16 *__restrict__ Alo, int64_t lda, const float *__restrict__ U,
    int64_t ldu, int64_t kdim, const float *W, float *Wout, float *__restrict__ beta, float *__restrict__ V,
    float *__restrict__ Bst, const uint8_t *__restrict__ codes, const float *__restrict__ c,
    const int *__restrict__ active, const DevParams<float> &q, int64_t ldp, int store_b, double *__restrict__ gpart,
    const GateArgs &ga, NodeCols ncl, int64_t bx, int64_t by, int64_t gx, float *red) {
    const int64_t m0 = bx * 32, n0 = by * 32;
    constexpr int E = 1024 / (64 * kWavesBf16);
    int sb[2], se[E];
    if (!tile_slots<32, 2, E, kWavesBf16>(ncl, n0, sb, se)) return;
    EpiIn<float> ei[E];
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * kWavesBf16;
        epi_load<float>(ei[t], se[t], n0 + (idx >> 5), m0 + (idx & 31), ldp, W, V, codes, c, active);
    }
    nt_tile_bf16<kWavesBf16>(Ahi, Alo, lda, U, ldu, kdim, m0, n0, sb, red);
    const bool est = gpart != nullptr;
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * kWavesBf16, n = idx >> 5, m = idx & 31;
        double e[5] = {0, 0, 0, 0, 0};
        if (ei[t].on)
            admm_update<float>(sum_waves<float, 32, 32, kWavesBf16>(red, n, m), ei[t], (int64_t)se[t] * ldp + m0 + m,
                               Wout, beta, V, Bst, q, store_b, est, ga, e);
        if (est) store_estimate<32>(e, m, se[t], gpart, gx, bx);
    }
}

__global__ __launch_bounds__(64 * kWavesBf16) void k_admm_xtu_bf16(
    const __bf16 *__restrict__ Ahi, const __bf16 *__restrict__ Alo, int64_t lda, const float *__restrict__ U,
    int64_t ldu, int64_t kdim, const float *W, float *Wout, float *__restrict__ beta, float *__restrict__ V,
    float *__restrict__ Bst, const uint8_t *__restrict__ codes, const float *__restrict__ c,
    const int *__restrict__ active, DevParams<float> q, int64_t ldp, int store_b, double *__restrict__ gpart,
    GateArgs ga, NodeCols ncl) {
    __shared__ float red[kWavesBf16 * Red<32, 32>::WS];
    xtu_bf16_tile(Ahi, Alo, lda, U, ldu, kdim, W, Wout, beta, V, Bst, codes, c, active, q, ldp, store_b, gpart, ga,
                  ncl, blockIdx.x, blockIdx.y, gridDim.x, red);
}

// Contraction over n of an anchored sweep in the BF16 split form (register
// tile): Q = z_a + Xh^T U with the BF16 pair, FP64 update, d = fl32(W - w_a).
__device__ __forceinline__ void xtu_anch_bf16_tile(
    const __bf16 *__restrict__ Ahi, const __bf16 *__restrict__ Alo, int64_t lda, const float *__restrict__ U,
    int64_t ldu, int64_t kdim, const double *__restrict__ Za, const double *__restrict__ Wa, double *__restrict__ W,
    double *__restrict__ beta, double *__restrict__ V, double *__restrict__ Bst, float *__restrict__ d,
    const uint8_t *__restrict__ codes, const double *__restrict__ c, const int *__restrict__ active,
    const DevParams<double> &q, int64_t ldp, int store_b, double *__restrict__ gpart, const GateArgs &ga,
    NodeCols ncl, int64_t bx, int64_t by, int64_t gx, float *red) {
    const int64_t m0 = bx * 32, n0 = by * 32;
    constexpr int E = 1024 / (64 * kWavesBf16);
    int sb[2], se[E];
    if (!tile_slots<32, 2, E, kWavesBf16>(ncl, n0, sb, se)) return;
    EpiIn<double> ei[E];
    double za[E], wa[E];
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * kWavesBf16;
        const int64_t col = n0 + (idx >> 5), j = m0 + (idx & 31), o = col_row(se[t], col) * ldp + j;
        epi_load<double>(ei[t], se[t], col, j, ldp, W, V, codes, c, active);
        za[t] = Za[o];
        wa[t] = Wa[o];
    }
    nt_tile_bf16<kWavesBf16>(Ahi, Alo, lda, U, ldu, kdim, m0, n0, sb, red);
    const bool est = gpart != nullptr;
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * kWavesBf16, n = idx >> 5, m = idx & 31;
        double e[5] = {0, 0, 0, 0, 0};
        if (ei[t].on) {
            const int64_t o = (int64_t)se[t] * ldp + m0 + m;
            const double Qv = za[t] + (double)sum_waves<float, 32, 32, kWavesBf16>(red, n, m);
            const double wn = admm_update<double>(Qv, ei[t], o, W, beta, V, Bst, q, store_b, est, ga, e);
            d[o] = (float)(wn - wa[t]);
        }
        if (est) store_estimate<32>(e, m, se[t], gpart, gx, bx);
    }
}

__global__ __launch_bounds__(64 * kWavesBf16) void k_admm_xtu_anch_bf16(
    const __bf16 *__restrict__ Ahi, const __bf16 *__restrict__ Alo, int64_t lda, const float *__restrict__ U,
    int64_t ldu, int64_t kdim, const double *__restrict__ Za, const double *__restrict__ Wa, double *__restrict__ W,
    double *__restrict__ beta, double *__restrict__ V, double *__restrict__ Bst, float *__restrict__ d,
    const uint8_t *__restrict__ codes, const double *__restrict__ c, const int *__restrict__ active,
    DevParams<double> q, int64_t ldp, int store_b, double *__restrict__ gpart, GateArgs ga, NodeCols ncl) {
    __shared__ float red[kWavesBf16 * Red<32, 32>::WS];
    xtu_anch_bf16_tile(Ahi, Alo, lda, U, ldu, kdim, Za, Wa, W, beta, V, Bst, d, codes, c, active, q, ldp, store_b,
                       gpart, ga, ncl, blockIdx.x, blockIdx.y, gridDim.x, red);
}

// Grouped launches of the BF16 split form (register tile, 8 waves): members as
// in the FP32 / FP64 groups, A given as its BF16 pair.
struct XwBfMember {
    const __bf16 *hi, *lo;
    const float *B;
    float *U;
    const int *cols;
    int64_t lda, ldb, ldu, kdim;
    int gx, tile0;
};

struct XtuBfMember {
    const __bf16 *hi, *lo;
    const float *U, *W, *c;
    float *Wout, *beta, *V, *Bst;
    const uint8_t *codes;
    const int *active, *cols;
    double *gpart;
    int64_t lda, ldu, kdim, ldp;
    int store_b, gx, tile0;
    DevParams<float> q;
    GateArgs ga;
};

struct AnchBfMember {
    const __bf16 *hi, *lo;
    const float *U;
    const double *Za, *Wa, *c;
    double *W, *beta, *V, *Bst;
    float *d;
    const uint8_t *codes;
    const int *active, *cols;
    double *gpart;
    int64_t lda, ldu, kdim, ldp;
    int store_b, gx, tile0;
    DevParams<double> q;
    GateArgs ga;
};

__global__ __launch_bounds__(64 * kWavesBf16) void k_gemm_xw_bf16_grp(Group<XwBfMember> g) {
    __shared__ float red[kWavesBf16 * Red<32, 32>::WS];
    const int b = blockIdx.x;
    const XwBfMember &d = g.m[group_member(g, b)];
    const int loc = b - d.tile0;
    xw_bf16_tile(d.hi, d.lo, d.lda, d.B, d.ldb, d.U, d.ldu, d.kdim, NodeCols{d.cols}, 0, loc % d.gx, loc / d.gx, 0, 1,
                 red);
}

__global__ __launch_bounds__(64 * kWavesBf16) void k_admm_xtu_bf16_grp(Group<XtuBfMember> g) {
    __shared__ float red[kWavesBf16 * Red<32, 32>::WS];
    const int b = blockIdx.x;
    const XtuBfMember &d = g.m[group_member(g, b)];
    const int loc = b - d.tile0;
    xtu_bf16_tile(d.hi, d.lo, d.lda, d.U, d.ldu, d.kdim, d.W, d.Wout, d.beta, d.V, d.Bst, d.codes, d.c, d.active, d.q,
                  d.ldp, d.store_b, d.gpart, d.ga, NodeCols{d.cols}, loc % d.gx, loc / d.gx, d.gx, red);
}

__global__ __launch_bounds__(64 * kWavesBf16) void k_admm_xtu_anch_bf16_grp(Group<AnchBfMember> g) {
    __shared__ float red[kWavesBf16 * Red<32, 32>::WS];
    const int b = blockIdx.x;
    const AnchBfMember &d = g.m[group_member(g, b)];
    const int loc = b - d.tile0;
    xtu_anch_bf16_tile(d.hi, d.lo, d.lda, d.U, d.ldu, d.kdim, d.Za, d.Wa, d.W, d.beta, d.V, d.Bst, d.d, d.codes, d.c,
                       d.active, d.q, d.ldp, d.store_b, d.gpart, d.ga, NodeCols{d.cols}, loc % d.gx, loc / d.gx, d.gx,
                       red);
}

static_assert(sizeof(Group<AnchBfMember>) <= 4096 && sizeof(Group<XtuBfMember>) <= 4096,
              "a group travels in the kernel arguments");

// ---------------------------------------------------------------------------
// FP8 storage (anchored sweeps only).  The folded operand is stored as FP8 e4m3
// codes with one FP32 scale per column, Xh[i][j] ~ q[i][j] s[j] with
// s[j] = max_i |Xh[i][j]| / 448, one byte per element in both layouts.  The
// products widen the codes to BF16 on load (exact: every e4m3 value is a BF16
// value) and multiply the node operand split into BF16 hi + lo:
//   U = Xh d   = q (s o d)      contraction over p: the operand is scaled on load
//   Q = Xh^T U = s o (q^T U)    contraction over n: the output is scaled
// so a product takes two BF16 MFMAs per block and a quarter of the FP32
// operand bytes.  The rounding of the codes (about 2^-4 relative) enters only
// through d = W - w_a: the anchor z_a = Xh^T Xh w_a is FP64, so the error of a
// sweep's product scales with the movement since the anchor and the iterates
// converge to the FP64 fixed point.
// ---------------------------------------------------------------------------

// 8 FP8 codes (one 8-byte word, code t in byte t) -> 8 BF16 values: each pair
// is widened to FP32 and the upper halves of the two patterns are packed (the
// truncation is exact for e4m3 values).
__device__ __forceinline__ bf16x8 fp8x8_to_bf16(uint2 v) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    u32x4 r;
#define L0L2_PAIR(w, hi)                                                                                  \
    __builtin_amdgcn_perm(__float_as_uint(__builtin_amdgcn_cvt_pk_f32_fp8((int)(w), hi)[1]),              \
                          __float_as_uint(__builtin_amdgcn_cvt_pk_f32_fp8((int)(w), hi)[0]), 0x07060302u)
    r[0] = L0L2_PAIR(v.x, false);
    r[1] = L0L2_PAIR(v.x, true);
    r[2] = L0L2_PAIR(v.y, false);
    r[3] = L0L2_PAIR(v.y, true);
#undef L0L2_PAIR
    return __builtin_bit_cast(bf16x8, r);
}

// 32 x 32 tile of C[m][n] = sum_k q[m][k] (sc[k] B[n][k]) (SCALE_B) or
// sum_k q[m][k] B[n][k] with q rows of FP8 codes (lda bytes) and B rows in FP32
// (split into BF16 hi, lo on load); chunks of 32 k split in pairs over WAVES
// waves with the branch-free two-stage loop of nt_tile.  Lane l reads the 8
// codes of row l%16 at k offset 8 (l/16) with one 8-byte load.  kdim must be a
// multiple of 64.
template <int WAVES, bool SCALE_B>
__device__ __forceinline__ void nt_tile_fp8(const uint8_t *__restrict__ qA, int64_t lda, const float *__restrict__ sc,
                                            const float *__restrict__ B, int64_t ldb, int64_t kdim, int64_t m0,
                                            int64_t n0, const int (&sb)[2], float *red, int64_t pr0 = 0,
                                            int64_t pr1 = -1) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int q = lane >> 4, r = lane & 15;
    const int64_t brow[2] = {col_row(sb[0], n0 + r), col_row(sb[1], n0 + 16 + r)};
    f32x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0, 0, 0, 0};
    // pairs [pr0, pr1) of 64 k (all of kdim by default), split over the waves
    if (pr1 < 0) pr1 = kdim / 64;
    const int64_t npr = pr1 - pr0;
    const int wu = __builtin_amdgcn_readfirstlane(w);
    const int64_t c0 = 2 * (pr0 + npr * wu / WAVES), c1 = 2 * (pr0 + npr * (wu + 1) / WAVES);
    uint2 av[2][2];
    float bv[2][2][8], sv[2][8];
    auto load = [&](int st, int64_t c) {
        for (int a = 0; a < 2; ++a)
            av[st][a] = *reinterpret_cast<const uint2 *>(qA + (m0 + 16 * a + r) * lda + 32 * c + 8 * q);
        for (int b = 0; b < 2; ++b) load8f(B + brow[b] * ldb + 32 * c + 8 * q, bv[st][b]);
        if (SCALE_B) load8f(sc + 32 * c + 8 * q, sv[st]);
        __builtin_amdgcn_sched_barrier(0);
    };
    auto compute = [&](int st) {
        const bf16x8 ah[2] = {fp8x8_to_bf16(av[st][0]), fp8x8_to_bf16(av[st][1])};
        for (int b = 0; b < 2; ++b) {
            float x[8];
            for (int t = 0; t < 8; ++t) x[t] = SCALE_B ? bv[st][b][t] * sv[st][t] : bv[st][b][t];
            bf16x8 bh, bl;
            split8(x, bh, bl);
            for (int a = 0; a < 2; ++a) {
                acc[a][b] = mfma16_bf16(ah[a], bh, acc[a][b]);
                acc[a][b] = mfma16_bf16(ah[a], bl, acc[a][b]);
            }
        }
    };
    if (c0 < c1) {
        load(0, c0);
        int64_t c = c0;
        for (; c + 2 < c1; c += 2) {
            load(1, c + 1);
            compute(0);
            __builtin_amdgcn_sched_barrier(0);
            load(0, c + 2);
            compute(1);
            __builtin_amdgcn_sched_barrier(0);
        }
        load(1, c + 1);
        compute(0);
        compute(1);
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int v = 0; v < 4; ++v) {
                int m = a * 16 + acc_row<float>(lane, v);
                int n = b * 16 + r;
                red[w * Red<32, 32>::WS + n * Red<32, 32>::LD + m] = acc[a][b][v];
            }
    __syncthreads();
}

// Contraction over p in FP8 storage: U[k][i] = sum_j q[i][j] s[j] d[k][j]; with
// gridDim.z = S > 1, slices of the range write partial products to U + z pstride
// as in k_gemm_xw.
__global__ __launch_bounds__(64 * kWavesBf16) void k_gemm_xw_fp8(const uint8_t *__restrict__ qA, int64_t lda,
                                                                 const float *__restrict__ sc,
                                                                 const float *__restrict__ B, int64_t ldb,
                                                                 float *__restrict__ U, int64_t ldu, int64_t kdim,
                                                                 NodeCols ncl, int64_t pstride) {
    __shared__ float red[kWavesBf16 * Red<32, 32>::WS];
    const int64_t m0 = (int64_t)blockIdx.x * 32, n0 = (int64_t)blockIdx.y * 32;
    constexpr int E = 1024 / (64 * kWavesBf16);
    int sb[2], se[E];
    if (!tile_slots<32, 2, E, kWavesBf16>(ncl, n0, sb, se)) return;
    const int64_t npr = kdim / 64, z = blockIdx.z, S = gridDim.z;
    U += pstride * z;
    nt_tile_fp8<kWavesBf16, true>(qA, lda, sc, B, ldb, kdim, m0, n0, sb, red, npr * z / S, npr * (z + 1) / S);
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * kWavesBf16, n = idx >> 5, m = idx & 31;
        if (se[t] >= 0) U[(int64_t)se[t] * ldu + m0 + m] = sum_waves<float, 32, 32, kWavesBf16>(red, n, m);
    }
}

// Contraction over n of an anchored sweep in FP8 storage: Q = z_a + s o (q^T U),
// FP64 update, d = fl32(W_new - w_a).
__global__ __launch_bounds__(64 * kWavesBf16) void k_admm_xtu_fp8(
    const uint8_t *__restrict__ qA, int64_t lda, const float *__restrict__ sc, const float *__restrict__ U,
    int64_t ldu, int64_t kdim, const double *__restrict__ Za, const double *__restrict__ Wa, double *__restrict__ W,
    double *__restrict__ beta, double *__restrict__ V, double *__restrict__ Bst, float *__restrict__ d,
    const uint8_t *__restrict__ codes, const double *__restrict__ c, const int *__restrict__ active,
    DevParams<double> q, int64_t ldp, int store_b, double *__restrict__ gpart, GateArgs ga, NodeCols ncl) {
    __shared__ float red[kWavesBf16 * Red<32, 32>::WS];
    const int64_t m0 = (int64_t)blockIdx.x * 32, n0 = (int64_t)blockIdx.y * 32;
    constexpr int E = 1024 / (64 * kWavesBf16);
    int sb[2], se[E];
    if (!tile_slots<32, 2, E, kWavesBf16>(ncl, n0, sb, se)) return;
    EpiIn<double> ei[E];
    double za[E], wa[E];
    float sj[E];
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * kWavesBf16;
        const int64_t col = n0 + (idx >> 5), j = m0 + (idx & 31), o = col_row(se[t], col) * ldp + j;
        epi_load<double>(ei[t], se[t], col, j, ldp, W, V, codes, c, active);
        za[t] = Za[o];
        wa[t] = Wa[o];
        sj[t] = sc[j];
    }
    nt_tile_fp8<kWavesBf16, false>(qA, lda, nullptr, U, ldu, kdim, m0, n0, sb, red);
    const bool est = gpart != nullptr;
#pragma unroll
    for (int t = 0; t < E; ++t) {
        const int idx = threadIdx.x + t * 64 * kWavesBf16, n = idx >> 5, m = idx & 31;
        double e[5] = {0, 0, 0, 0, 0};
        if (ei[t].on) {
            const int64_t o = (int64_t)se[t] * ldp + m0 + m;
            const double Qv = za[t] + (double)sj[t] * (double)sum_waves<float, 32, 32, kWavesBf16>(red, n, m);
            const double wn = admm_update<double>(Qv, ei[t], o, W, beta, V, Bst, q, store_b, est, ga, e);
            d[o] = (float)(wn - wa[t]);
        }
        if (est) store_estimate<32>(e, m, se[t], gpart);
    }
}

// LDS-staged tile of the FP8 form (4 waves, 2 x 2; TM = 32 WM, TN = 32 WN).  A k
// chunk of 32 stages, per row, the 32 code bytes of A (rows 32 bytes apart: the
// 8-byte fragment reads of 16 rows x 4 k offsets cover 512 contiguous bytes)
// and the BF16 hi and lo terms of B (its FP32 values split as they are staged;
// rows of 2 x 64 bytes padded to 144 as in the BF16 tile); lane l reads the 8
// codes of row l%16 at k offset 8 (l/16) and widens them, and the matching hi
// and lo terms of B.  SCALE_B (the contraction over p) multiplies B by the
// column scales s_k as it is loaded, before the split, as the register tile
// does; the contraction over n scales its output rows instead.
template <int WM, int WN>
struct LdsTileF8 {
    static constexpr int TM = 32 * WM, TN = 32 * WN;
    static constexpr int ROWA = 32, ROWB = 144;                // bytes per staged row
    static constexpr int PA = TM * 2, NA = (PA + 255) / 256;   // 16-byte parts of the A slab
    static constexpr int NB = TN * 8 / 256;
    static constexpr int STAGE = TM * ROWA + TN * ROWB;        // bytes per buffer
};

template <int WM, int WN, bool SCALE_B>
__device__ __forceinline__ void lds_tile_fp8(const uint8_t *__restrict__ qA, int64_t lda, const float *__restrict__ sc,
                                             const float *__restrict__ B, int64_t ldb, int64_t kdim, int64_t m0,
                                             int64_t n0, const NodeCols &ncl, unsigned char *smem,
                                             f32x4 (&acc)[WM][WN]) {
    typedef LdsTileF8<WM, WN> L;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int q = lane >> 4, r = lane & 15;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    // staged 16-byte part e of this thread: A row idx / 2, part idx % 2 (only
    // idx < PA); B row idx / 8, part idx % 8
    const unsigned char *ga[L::NA];
    const unsigned char *gb[L::NB];
    int la[L::NA], lb[L::NB], pb[L::NB];
    bool ha[L::NA];
#pragma unroll
    for (int e = 0; e < L::NA; ++e) {
        const int idx = tid + 256 * e, row = (idx < L::PA ? idx : 0) >> 1, part = idx & 1;
        ha[e] = idx < L::PA;
        ga[e] = qA + (m0 + row) * lda + 16 * part;
        la[e] = row * L::ROWA + 16 * part;
    }
#pragma unroll
    for (int e = 0; e < L::NB; ++e) {
        const int idx = tid + 256 * e, row = idx >> 3, part = idx & 7;
        gb[e] = reinterpret_cast<const unsigned char *>(B + col_row(col_slot(ncl, n0 + row), n0 + row) * ldb) +
                16 * part;
        lb[e] = L::TM * L::ROWA + row * L::ROWB + 8 * part;
        pb[e] = 4 * part;
    }
    float4 va[L::NA], vb[L::NB];
    // chunk c covers 32 k: 32 code bytes, 128 bytes of FP32 (times the 4 scales
    // of its k when SCALE_B)
#define L0L2_GLOADF(c)                                                                                       \
    _Pragma("unroll") for (int e = 0; e < L::NA; ++e) va[e] = *reinterpret_cast<const float4 *>(ga[e] + 32 * (c)); \
    _Pragma("unroll") for (int e = 0; e < L::NB; ++e) {                                                      \
        vb[e] = *reinterpret_cast<const float4 *>(gb[e] + 128 * (c));                                         \
        if (SCALE_B) {                                                                                        \
            const float4 s4 = *reinterpret_cast<const float4 *>(sc + 32 * (c) + pb[e]);                       \
            vb[e].x *= s4.x;                                                                                  \
            vb[e].y *= s4.y;                                                                                  \
            vb[e].z *= s4.z;                                                                                  \
            vb[e].w *= s4.w;                                                                                  \
        }                                                                                                     \
    }
#define L0L2_SSTOREF(st)                                                                                     \
    _Pragma("unroll") for (int e = 0; e < L::NA; ++e) if (ha[e])                                              \
        *reinterpret_cast<float4 *>(smem + (st) * L::STAGE + la[e]) = va[e];                                  \
    _Pragma("unroll") for (int e = 0; e < L::NB; ++e) {                                                      \
        bf16x4 h4, l4;                                                                                       \
        split4(vb[e], h4, l4);                                                                               \
        *reinterpret_cast<bf16x4 *>(smem + (st) * L::STAGE + lb[e]) = h4;                                     \
        *reinterpret_cast<bf16x4 *>(smem + (st) * L::STAGE + lb[e] + 64) = l4;                                \
    }
    const int64_t nch = kdim / 32;
    L0L2_GLOADF(0)
    L0L2_SSTOREF(0)
    __syncthreads();
    for (int64_t c = 0; c < nch; ++c) {
        const int st = (int)(c & 1);
        const int64_t cn = c + 1 < nch ? c + 1 : c;
        L0L2_GLOADF(cn)
        const unsigned char *sa = smem + st * L::STAGE;
        bf16x8 ah[WM], bh[WN], bl[WN];
#pragma unroll
        for (int i = 0; i < WM; ++i)
            ah[i] = fp8x8_to_bf16(*reinterpret_cast<const uint2 *>(sa + (wm * 16 * WM + 16 * i + r) * L::ROWA + 8 * q));
#pragma unroll
        for (int j = 0; j < WN; ++j) {
            const unsigned char *row = sa + L::TM * L::ROWA + (wn * 16 * WN + 16 * j + r) * L::ROWB;
            bh[j] = *reinterpret_cast<const bf16x8 *>(row + 16 * q);
            bl[j] = *reinterpret_cast<const bf16x8 *>(row + 64 + 16 * q);
        }
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
            for (int j = 0; j < WN; ++j) {
                acc[i][j] = mfma16_bf16(ah[i], bh[j], acc[i][j]);
                acc[i][j] = mfma16_bf16(ah[i], bl[j], acc[i][j]);
            }
        L0L2_SSTOREF(st ^ 1)
        __syncthreads();
    }
#undef L0L2_GLOADF
#undef L0L2_SSTOREF
}

// Contraction over p in FP8 storage, LDS-staged tile: U[k][i] = sum_j q[i][j]
// s[j] d[k][j].  With gridDim.z = S > 1, slice z takes the chunks
// [nch z / S, nch (z + 1) / S) of 32 k (the launcher keeps S <= nch, so none is
// empty) and writes its partial product to U + z pstride.
template <int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm_xw_fp8_lds(const uint8_t *__restrict__ qA, int64_t lda,
                                                         const float *__restrict__ sc, const float *__restrict__ B,
                                                         int64_t ldb, float *__restrict__ U, int64_t ldu,
                                                         int64_t kdim, NodeCols ncl, int64_t pstride) {
    typedef LdsTileF8<WM, WN> L;
    __shared__ __align__(16) unsigned char smem[2 * L::STAGE];
    const int64_t m0 = (int64_t)blockIdx.x * L::TM, n0 = (int64_t)blockIdx.y * L::TN;
    if (col_slot(ncl, n0) < 0) return;
    const int64_t nch = kdim / 32, z = blockIdx.z, S = gridDim.z;
    const int64_t c0 = nch * z / S, c1 = nch * (z + 1) / S;
    U += pstride * z;
    f32x4 acc[WM][WN];
    lds_tile_fp8<WM, WN, true>(qA + 32 * c0, lda, sc + 32 * c0, B + 32 * c0, ldb, 32 * (c1 - c0), m0, n0, ncl, smem,
                               acc);
    typedef LdsEpi<float, WM, WN> E;
    constexpr int NP = E::passes(sizeof(smem));
    static_assert(NP > 0, "epilogue staging does not fit");
    constexpr int PN = L::TN / NP;
    float *buf = reinterpret_cast<float *>(smem);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int pass = 0; pass < NP; ++pass) {
        const int cc = pass * PN;
        __syncthreads();
        acc_stage<float, WM, WN>(acc, buf, cc, PN);
        __syncthreads();
        for (int t = 0; t < PN / 4; ++t) {
            const int nl = cc + w + 4 * t, slot = col_slot(ncl, n0 + nl);
            if (slot < 0) continue;
#pragma unroll
            for (int h = 0; h < E::H; ++h)
                U[(int64_t)slot * ldu + m0 + lane + 64 * h] = buf[(nl - cc) * E::LD + lane + 64 * h];
        }
    }
}

// Contraction over n of an anchored sweep in FP8 storage, LDS-staged tile:
// Q = z_a + s o (q^T U), FP64 update, d = fl32(W_new - w_a), with the
// node-major LDS epilogue of the other LDS tiles.
template <int WM, int WN>
__global__ __launch_bounds__(256) void k_admm_xtu_fp8_lds(
    const uint8_t *__restrict__ qA, int64_t lda, const float *__restrict__ sc, const float *__restrict__ U,
    int64_t ldu, int64_t kdim, const double *__restrict__ Za, const double *__restrict__ Wa, double *__restrict__ W,
    double *__restrict__ beta, double *__restrict__ V, double *__restrict__ Bst, float *__restrict__ d,
    const uint8_t *__restrict__ codes, const double *__restrict__ c, const int *__restrict__ active,
    DevParams<double> q, int64_t ldp, int store_b, double *__restrict__ gpart, GateArgs ga, NodeCols ncl) {
    typedef LdsTileF8<WM, WN> L;
    __shared__ __align__(16) unsigned char smem[2 * L::STAGE];
    const int64_t m0 = (int64_t)blockIdx.x * L::TM, n0 = (int64_t)blockIdx.y * L::TN;
    if (col_slot(ncl, n0) < 0) return;
    f32x4 acc[WM][WN];
    lds_tile_fp8<WM, WN, false>(qA, lda, nullptr, U, ldu, kdim, m0, n0, ncl, smem, acc);
    const bool est = gpart != nullptr;
    typedef LdsEpi<float, WM, WN> E;
    constexpr int NP = E::passes(sizeof(smem));
    static_assert(NP > 0, "epilogue staging does not fit");
    constexpr int PN = L::TN / NP;
    float *buf = reinterpret_cast<float *>(smem);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float sj[E::H];
#pragma unroll
    for (int h = 0; h < E::H; ++h) sj[h] = sc[m0 + lane + 64 * h];
    for (int pass = 0; pass < NP; ++pass) {
        const int c0 = pass * PN;
        __syncthreads();
        acc_stage<float, WM, WN>(acc, buf, c0, PN);
        __syncthreads();
        for (int t = 0; t < PN / 4; ++t) {
            const int nl = c0 + w + 4 * t, slot = col_slot(ncl, n0 + nl);
            EpiIn<double> ei[E::H];
            double za[E::H], wa[E::H];
            epi_load_row<double, E::H>(ei, slot, n0 + nl, m0, ldp, W, V, codes, c, active);
#pragma unroll
            for (int h = 0; h < E::H; ++h) {
                const int64_t o = col_row(slot, n0 + nl) * ldp + m0 + lane + 64 * h;
                za[h] = Za[o];
                wa[h] = Wa[o];
            }
            double e[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int h = 0; h < E::H; ++h) {
                if (!ei[h].on) continue;
                const int m = lane + 64 * h;
                const int64_t o = (int64_t)slot * ldp + m0 + m;
                double ev[5] = {0, 0, 0, 0, 0};
                const double Qv = za[h] + (double)sj[h] * (double)buf[(nl - c0) * E::LD + m];
                const double wn = admm_update<double>(Qv, ei[h], o, W, beta, V, Bst, q, store_b, est, ga, ev);
                d[o] = (float)(wn - wa[h]);
#pragma unroll
                for (int u = 0; u < 5; ++u) e[u] += ev[u];
            }
            if (est) {
                wave_sum5(e);
                if (lane == 0 && slot >= 0)
                    for (int u = 0; u < 5; ++u) gpart[((int64_t)slot * gridDim.x + blockIdx.x) * 5 + u] = e[u];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Gap check (FP64)
// ---------------------------------------------------------------------------
// Sum over the 64 lanes of a wave (xor butterfly: every lane gets the same value).
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// First kernel of the gap check: with the original X (row-major copy, FP64)
// and the node iterates b (grid z = 0) and beta (z = 1) of type T, forms the
// 16 BM x 16 BN tile of X b^T (X beta^T) for the nodes of the check list and,
// in the epilogue, r = y - X b (stored in R) with the per-(node, 32-row tile)
// sums of ||r||^2, y^T r, |y|^T |r| (z = 0) or ||y - X beta||^2 (z = 1) in
// rpart[(node * ntr + tile) * 4 + {0, 1, 2 | 3}], ntr = rows / 32.  Wider node
// tiles read each X panel fewer times, for large batches.
template <class T, int BM, int BN, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_check_xr(const double *__restrict__ XR, int64_t ldx,
                                                         const T *__restrict__ B, const T *__restrict__ beta,
                                                         int64_t ldb, int64_t kdim, const double *__restrict__ y,
                                                         double *__restrict__ R, int64_t ldr,
                                                         double *__restrict__ rpart, NodeCols ncl) {
    constexpr int TM = 16 * BM, TN = 16 * BN;
    static_assert(TM == 32 || TM == 64, "row tiles of 32 or 64");
    __shared__ double red[WAVES * Red<TM, TN>::WS];
    const bool with_b = blockIdx.z == 0;
    const int64_t m0 = (int64_t)blockIdx.x * TM, n0 = (int64_t)blockIdx.y * TN;
    constexpr int E = TM * TN / (64 * WAVES);
    static_assert(E * 64 * WAVES == TM * TN, "tile elements per thread");
    int sb[BN], se[E];
    if (!tile_slots<TM, BN, E, WAVES>(ncl, n0, sb, se)) return;
    nt_tile<double, T, double, BM, BN, WAVES>(XR, ldx, with_b ? B : beta, ldb, kdim, m0, n0, sb, red);
    const int64_t ntr = (int64_t)gridDim.x * (TM / 32);
#pragma unroll
    for (int t = 0; t < E; ++t) {
        // 32 consecutive lanes hold 32 rows of one node: one 32-row tile
        const int idx = threadIdx.x + t * 64 * WAVES, n = idx / TM, m = idx % TM;
        const bool live = se[t] >= 0;
        const int64_t node = se[t], i = m0 + m;
        const double yi = y[i];
        const double rv = yi - sum_waves<double, TM, TN, WAVES>(red, n, m);
        double e0, e1 = 0.0, e2 = 0.0;
        if (with_b) {
            if (live) R[node * ldr + i] = rv;
            e0 = rv * rv;
            e1 = yi * rv;
            e2 = fabs(yi) * fabs(rv);
        } else {
            e0 = rv * rv;
        }
        for (int off = 1; off < 32; off <<= 1) {
            e0 += __shfl_xor(e0, off);
            e1 += __shfl_xor(e1, off);
            e2 += __shfl_xor(e2, off);
        }
        if ((m & 31) == 0 && live) {
            double *d = rpart + (node * ntr + (i >> 5)) * 4;
            if (with_b) {
                d[0] = e0;
                d[1] = e1;
                d[2] = e2;
            } else {
                d[3] = e0;
            }
        }
    }
}

struct DualArgs {
    double l0, l2, M, s, two_M_l2, four_l2, l2_M2, psi_lin, gamma_n;
    int free_quad;
    int64_t p;
};

// g = X^T r per (node, coordinate) with the per-tile sums of the upper bounds
// of nu_i(|g_i|) and of psi_i(beta_i) over 32-coordinate tiles:
// part[(k * ntile + tile) * 3 + {0,1,2}] = sum nu+, sum |nu+|, sum psi,
// ntile = padded p / 32.  The output tile is 16 BM coordinates x 16 BN nodes.
template <class T, int BM, int BN, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_dual_xtr(
    const double *__restrict__ A, int64_t lda, const double *__restrict__ R, int64_t ldr, int64_t kdim,
    const uint8_t *__restrict__ codes, const T *__restrict__ beta, const double *__restrict__ colnrm,
    const double *__restrict__ rpart, int64_t ntr, const int *__restrict__ active, double *__restrict__ part,
    int64_t ldp, DualArgs da, NodeCols ncl) {
    constexpr int TM = 16 * BM, TN = 16 * BN;
    __shared__ double red[WAVES * Red<TM, TN>::WS];
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * TM, n0 = (int64_t)blockIdx.y * TN;
    constexpr int E = TM * TN / (64 * WAVES);
    // TPN consecutive threads per node; thread t takes node t / TPN and the CPT
    // coordinates from CPT (t % TPN), all in one 32-coordinate tile (TPH
    // threads per tile)
    constexpr int TPN = 64 * WAVES / TN, CPT = TM / TPN, TPH = TPN / (TM / 32);
    static_assert(TPN * CPT == TM && TPN <= 64 && TPH >= 1 && CPT <= 32, "threads per node");
    int sb[BN], se[E];
    const int n = tid / TPN, jl = (tid % TPN) * CPT;
    const int slot = col_slot(ncl, n0 + n);
    if (!tile_slots<TM, BN, E, WAVES>(ncl, n0, sb, se)) return;
    nt_tile<double, double, double, BM, BN, WAVES>(A, lda, R, ldr, kdim, m0, n0, sb, red);
    const bool live = slot >= 0;
    const int64_t node = col_row(slot, n0 + n);   // rows read for an idle column are valid and unused
    // ||r||^2 of the node from the row-tile sums of the first check kernel
    double rr = 0.0;
    for (int64_t t = tid % TPN; t < ntr; t += TPN) rr += rpart[(node * ntr + t) * 4];
    for (int off = 1; off < TPN; off <<= 1) rr += __shfl_xor(rr, off);
    double snu = 0, sanu = 0, spsi = 0;
    const bool act = live && active[node] != 0;
    if (act) {
        const double nr = sqrt(rr);
        for (int e = 0; e < CPT; ++e) {
            int64_t j = m0 + jl + e;
            if (j >= da.p) continue;
            double g = sum_waves<double, TM, TN, WAVES>(red, n, jl + e);
            uint8_t code = codes[node * ldp + j];
            double ej = 2.0 * da.gamma_n * colnrm[j] * nr;
            double val = nu_upper(fabs(g), ej, code, da.l0, da.l2, da.M, da.two_M_l2, da.four_l2, da.l2_M2,
                                  da.free_quad);
            snu += val;
            sanu += fabs(val);
            spsi += psi_val((double)beta[node * ldp + j], code, da.l0, da.l2, da.s, da.free_quad, da.psi_lin);
        }
    }
    for (int off = 1; off < TPH; off <<= 1) {
        snu += __shfl_xor(snu, off);
        sanu += __shfl_xor(sanu, off);
        spsi += __shfl_xor(spsi, off);
    }
    if (tid % TPH == 0 && act) {
        const int64_t ntile = (int64_t)gridDim.x * (TM / 32);
        double *pp = part + (node * ntile + ((m0 + jl) >> 5)) * 3;
        pp[0] = snu;
        pp[1] = sanu;
        pp[2] = spsi;
    }
}

struct FinArgs {
    double gamma_n2, gamma_p, tol, switch_tol;
    int64_t K, ntile, ntr;
    int mode;    // mode 0: solve (gap test), 1: bound only
    int budget;  // > 0: a node that has done this many sweeps since it started retires (status 1)
};

// One wave per node slot: LB = (q - sum nu+) - margin (Prop. 1 plus the
// rounding margin) and, in mode 0, P(beta) = 1/2 ||y - X beta||^2 + sum psi
// and the gap test, for the active nodes that were checked (all of them, or
// those the gap estimate flagged in needs).  In mode 0 every node that stays
// active is appended to the next active list (nlist, *ncount) and counted in
// counter[0], and in counter[1] when its gap is above switch_tol (the exact
// gap, or the estimate gest, a lower bound of it, for the nodes left out of
// the check).  Appends and counts are integer atomics: the counts are exact in
// any order, and the order of the list does not change any node's arithmetic.
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ rpart, const double *__restrict__ part,
                                                  int *__restrict__ active, int *__restrict__ status,
                                                  int *__restrict__ iters, double *__restrict__ lb,
                                                  double *__restrict__ primal, int *__restrict__ counter,
                                                  int *__restrict__ nlist, int *__restrict__ ncount,
                                                  const int *__restrict__ sweep_no, FinArgs fa,
                                                  const int *__restrict__ needs, const double *__restrict__ gest,
                                                  const int *__restrict__ start, int *__restrict__ dlist) {
    const int lane = threadIdx.x & 63;
    const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= fa.K || !active[k]) return;
    // a retired node (converged, or at its sweep budget) is listed for the host
    auto retire = [&](int st) {
        status[k] = st;
        active[k] = 0;
        dlist[atomicAdd(&counter[2], 1)] = (int)k;
    };
    auto keep = [&](bool above) {
        nlist[atomicAdd(ncount, 1)] = (int)k;
        atomicAdd(&counter[0], 1);
        if (above) atomicAdd(&counter[1], 1);
    };
    if (needs && !needs[k]) {
        if (lane == 0 && fa.mode == 0) keep(gest[k] > fa.switch_tol);
        return;
    }
    const double u = 1.1102230246251565e-16;
    double rr = 0, yr = 0, ayr = 0, rbrb = 0, snu = 0, sanu = 0, spsi = 0;
    const double *rk = rpart + k * fa.ntr * 4;
    for (int64_t t = lane; t < fa.ntr; t += 64) {
        rr += rk[t * 4 + 0];
        yr += rk[t * 4 + 1];
        ayr += rk[t * 4 + 2];
        if (fa.mode == 0) rbrb += rk[t * 4 + 3];
    }
    const double *pk = part + k * fa.ntile * 3;
    for (int64_t t = lane; t < fa.ntile; t += 64) {
        snu += pk[t * 3 + 0];
        sanu += pk[t * 3 + 1];
        spsi += pk[t * 3 + 2];
    }
    rr = wave_sum(rr);
    yr = wave_sum(yr);
    ayr = wave_sum(ayr);
    rbrb = wave_sum(rbrb);
    snu = wave_sum(snu);
    sanu = wave_sum(sanu);
    spsi = wave_sum(spsi);
    if (lane != 0) return;
    const double qv = -0.5 * rr + yr;
    const double margin =
        2.0 * fa.gamma_n2 * (0.5 * rr + ayr) + 2.0 * fa.gamma_p * sanu + 4.0 * u * (fabs(qv) + fabs(snu));
    const double LB = (qv - snu) - margin;
    lb[k] = LB;
    if (fa.mode == 1) return;
    const double P = 0.5 * rbrb + spsi;
    primal[k] = P;
    const int done = *sweep_no - start[k];
    iters[k] = done;
    const double den = fabs(P) > 1e-300 ? fabs(P) : 1e-300;
    if ((P - LB) / den <= fa.tol) {
        retire(0);
    } else if (fa.budget > 0 && done >= fa.budget) {
        retire(1);
    } else {
        status[k] = 1;
        keep((P - LB) / den > fa.switch_tol);
    }
}

// The next active list becomes the current one, with -1 past its nodes, and
// the check list is emptied (all -1) for the next gap estimate (one workgroup).
__global__ __launch_bounds__(256) void k_list_commit(const int *__restrict__ nlist, const int *__restrict__ ncount,
                                                     int *__restrict__ list, int *__restrict__ clist, int64_t Kp) {
    const int n = *ncount;
    for (int64_t i = threadIdx.x; i < Kp; i += 256) {
        list[i] = i < n ? nlist[i] : -1;
        clist[i] = -1;
    }
}

struct GateFin {
    double yy, tol;
    int64_t K, ntile;
    int budget;   // > 0: nodes at their sweep budget go to the exact check whatever the estimate
    int skip;     // 1: no node goes to the exact check (the estimate alone steers the switch)
};

// Gap estimate per node (one wave each) from the per-tile sums of the last
// sweep's epilogue: gest[k] = 1 - D / P_low.  A node needs the exact check
// unless P_low > 0 and P_low - D > 2 tol P_low: then its P(beta) is at least
// P_low and its rigorous LB at most D (up to rounding), so the check's
// relative gap 1 - LB / P(beta) is at least gest[k] and the check cannot accept
// it.  needs[k] flags the node; the nodes that need the check are appended to
// the check list (clist, gate[0]) with integer atomics.
__global__ __launch_bounds__(256) void k_gate(const double *__restrict__ gpart, const int *__restrict__ active,
                                              int *__restrict__ needs, double *__restrict__ gest,
                                              int *__restrict__ clist, int *__restrict__ gate, GateFin gf,
                                              const int *__restrict__ sweep_no, const int *__restrict__ start) {
    const int lane = threadIdx.x & 63;
    const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= gf.K || !active[k]) return;
    double e[5] = {0, 0, 0, 0, 0};
    const double *pk = gpart + k * gf.ntile * 5;
    for (int64_t t = lane; t < gf.ntile; t += 64)
        for (int i = 0; i < 5; ++i) e[i] += pk[t * 5 + i];
    for (int i = 0; i < 5; ++i) e[i] = wave_sum(e[i]);
    if (lane == 0) {
        const double rr = gf.yy - 2.0 * e[0] + e[1];
        const double D = -0.5 * rr + (gf.yy - e[0]) - e[2];
        const double Pl = 0.5 * rr - e[3] + e[4];
        const bool spent = gf.budget > 0 && *sweep_no - start[k] >= gf.budget;
        const bool far = !spent && (gf.skip || (Pl > 0.0 && (Pl - D) > 2.0 * gf.tol * Pl));
        needs[k] = far ? 0 : 1;
        gest[k] = Pl > 0.0 ? (Pl - D) / Pl : INFINITY;
        if (!far) clist[atomicAdd(&gate[0], 1)] = (int)k;
    }
}

// Ladder step: FP64 copies of the FP32 node state, W64 = c + rho beta - V.
__global__ void k_promote(const float *__restrict__ beta, const float *__restrict__ V, double *__restrict__ beta64,
                          double *__restrict__ V64, double *__restrict__ W64, const double *__restrict__ c,
                          double rho, int64_t pp, int64_t total) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        double b = (double)beta[idx], v = (double)V[idx];
        beta64[idx] = b;
        V64[idx] = v;
        W64[idx] = c[idx % pp] + rho * b - v;
    }
}

__global__ void k_demote(const double *__restrict__ beta64, const double *__restrict__ V64, float *__restrict__ beta,
                         float *__restrict__ V, int64_t total) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        beta[idx] = (float)beta64[idx];
        V[idx] = (float)V64[idx];
    }
}

unsigned grid1d(int64_t total) { return (unsigned)std::min<int64_t>((total + 255) / 256, 65536); }

// The arrays one sweep works on, in the arithmetic type T of the sweep.
template <class T>
struct Sweep {
    const T *Xh;   // np x pp folded operand, column-major (column stride ldc)
    const T *XhR;  // the same, row-major (row stride ldr)
    const T *c;    // ldp entries
    T *W, *beta, *V, *B;   // node-state rows of stride ldp
    T *U;          // ADMM product rows of stride ldu
    int64_t ldc, ldr, ldu, ldp;
};

Sweep<double> sweep64(l0l2_ctx *ctx) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    if (in.prec == L0L2_FP64)
        return {in.Xh.as<double>(), in.XhRw.as<double>(), in.c64.as<double>(), ws.W.as<double>(),
                ws.beta.as<double>(), ws.V.as<double>(), ws.B.as<double>(), ws.U.as<double>(),
                in.ldx, in.ldxr, in.ldu, in.ldp};
    return {in.Xh64.as<double>(), in.Xh64R.as<double>(), in.c64.as<double>(), ws.W64.as<double>(),
            ws.beta64.as<double>(), ws.V64.as<double>(), ws.B64.as<double>(), ws.U64.as<double>(),
            in.ldx, in.ldxr, in.ldu64, in.ldp};
}

// FP32 state arrays (the FP32 mode's operand; in BF16 mode Xh is the BF16 pair
// and is not read through this struct).
Sweep<float> sweep32(l0l2_ctx *ctx) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    const bool f32 = in.prec == L0L2_FP32;
    return {f32 ? in.Xh.as<float>() : nullptr, f32 ? in.XhRw.as<float>() : nullptr, in.cst.as<float>(),
            ws.W.as<float>(), ws.beta.as<float>(), ws.V.as<float>(), ws.B.as<float>(), ws.U.as<float>(),
            in.ldw, in.ldwr, in.ldu, in.ldp};
}

template <class T> constexpr int prof_xw();
template <> constexpr int prof_xw<float>() { return PROF_GEMM_XW_F32; }
template <> constexpr int prof_xw<double>() { return PROF_GEMM_XW_F64; }
template <class T> constexpr int prof_xtu();
template <> constexpr int prof_xtu<float>() { return PROF_ADMM_XTU_F32; }
template <> constexpr int prof_xtu<double>() { return PROF_ADMM_XTU_F64; }

// ---------------------------------------------------------------------------
// Host drivers
// ---------------------------------------------------------------------------
// Tile shapes of the sweep contractions: output tile TM x TN (rows x nodes) and
// waves per workgroup.  Shapes 0-8 are register tiles whose waves split the
// contraction range (FP64 keeps at most 8 waves on the 32 x 32 tile: LDS for
// the cross-wave reduction); shapes 9-11 are LDS-staged tiles (4 waves, 2 x 2).
// Shapes 12-17 serve the contraction over p only and cut its range into
// slices: 12, 13, 17 = the 128 x 128 LDS-staged tile in 2, 4 or 8 slices; 14, 15
// = the 16 x 16 register tile (4 waves) in 4 or 8 slices; 16 = the 32 x 32
// register tile (4 waves) in 4 slices.
constexpr int kShapes = 12, kShapesXw = 18;
constexpr int kTileTM[kShapesXw] = {32, 32, 32, 16, 32, 16, 64, 32, 64, 64, 128, 128, 128, 128, 16, 16, 32, 128};
constexpr int kTileTN[kShapesXw] = {32, 32, 32, 32, 16, 16, 32, 64, 64, 64, 64, 128, 128, 128, 16, 16, 32, 128};
constexpr int kTileW[kShapesXw] = {4, 8, 16, 8, 8, 4, 8, 8, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4};
constexpr int kSplit[kShapesXw] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 4, 4, 8, 4, 8};
constexpr int kMaxSplit = 8;
int split_of(int v) { return kSplit[v]; }

// Partial-product buffer of the sliced shapes.  A slice writes node slot k's
// partial row at k ldu, and the slots of a live bucket's columns range over the
// whole padded batch (not only the bucket's width), so each slice spans `rows`
// node rows: the workspace's node capacity.
struct SplitBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int64_t rows = 0;
};

// A shape fits a padded batch when its node tile divides it (rows are padded to
// multiples of 128).
bool shape_fits(int v, int64_t Kp) { return Kp % kTileTN[v] == 0; }

template <class TA, class TB, class TC>
void launch_xw(int v, hipStream_t s, const TA *A, int64_t lda, const TB *B, int64_t ldb, TC *U, int64_t ldu,
               int64_t rows, int64_t Kp, int64_t kdim, NodeCols ncl = NodeCols{nullptr}, SplitBuf sk = SplitBuf{}) {
    if (sizeof(TC) == 8 && v == 2) v = 1;
    if (v < 0 || v >= kShapesXw || !shape_fits(v, Kp)) fail(L0L2_E_INVALID, "tile shape does not fit the batch");
    dim3 g((unsigned)(rows / kTileTM[v]), (unsigned)(Kp / kTileTN[v]));
    dim3 b((unsigned)(64 * kTileW[v]));
#define L0L2_XW(PBM, PBN, PW) \
    hipLaunchKernelGGL((k_gemm_xw<TA, TB, TC, PBM, PBN, PW>), g, b, 0, s, A, lda, B, ldb, U, ldu, kdim, ncl, (int64_t)0)
#define L0L2_XWL(WM, WN) \
    hipLaunchKernelGGL((k_gemm_xw_lds<TC, WM, WN>), g, b, 0, s, (const TC *)A, lda, (const TC *)B, ldb, U, ldu, kdim, \
                       ncl, (int64_t)0)
    if (v >= kShapes) {
        const int S = split_of(v);
        const int64_t pstride = sk.rows * ldu;
        if (sk.rows < Kp || (size_t)S * pstride * sizeof(TC) > sk.bytes) fail(L0L2_E_INVALID, "split buffer too small");
        TC *P = static_cast<TC *>(sk.ptr);
        const dim3 gs(g.x, g.y, (unsigned)S);
        if (v <= 13 || v == 17) {
            if (!std::is_same<TA, TC>::value || !std::is_same<TB, TC>::value)
                fail(L0L2_E_INVALID, "LDS-staged tiles take one operand type");
            hipLaunchKernelGGL((k_gemm_xw_lds<TC, 4, 4>), gs, b, 0, s, (const TC *)A, lda, (const TC *)B, ldb, P, ldu,
                               kdim, ncl, pstride);
        } else if (v <= 15) {
            hipLaunchKernelGGL((k_gemm_xw<TA, TB, TC, 1, 1, 4>), gs, b, 0, s, A, lda, B, ldb, P, ldu, kdim, ncl,
                               pstride);
        } else {
            hipLaunchKernelGGL((k_gemm_xw<TA, TB, TC, 2, 2, 4>), gs, b, 0, s, A, lda, B, ldb, P, ldu, kdim, ncl,
                               pstride);
        }
        hipLaunchKernelGGL(k_splitk_sum<TC>, dim3((unsigned)((rows + 255) / 256), (unsigned)Kp), dim3(256), 0, s,
                           (const TC *)P, pstride, S, U, ldu, rows, ncl);
        return;
    }
    if (v >= 9) {
        if (!std::is_same<TA, TC>::value || !std::is_same<TB, TC>::value)
            fail(L0L2_E_INVALID, "LDS-staged tiles take one operand type");
        switch (v) {
            case 9: L0L2_XWL(2, 2); break;
            case 10: L0L2_XWL(4, 2); break;
            default: L0L2_XWL(4, 4); break;
        }
        return;
    }
    switch (v) {
        case 0: L0L2_XW(2, 2, 4); break;
        case 1: L0L2_XW(2, 2, 8); break;
        case 2: L0L2_XW(2, 2, (sizeof(TC) == 8 ? 8 : 16)); break;
        case 3: L0L2_XW(1, 2, 8); break;
        case 4: L0L2_XW(2, 1, 8); break;
        case 5: L0L2_XW(1, 1, 4); break;
        case 6: L0L2_XW(4, 2, 8); break;
        case 7: L0L2_XW(2, 4, 8); break;
        default: L0L2_XW(4, 4, 4); break;
    }
#undef L0L2_XW
#undef L0L2_XWL
}

template <class T>
void launch_xtu(int v, hipStream_t s, const Sweep<T> &sw, int64_t np, int64_t pp, int64_t Kp, const uint8_t *codes,
                const int *active, const DevParams<T> &q, int store_b, double *gpart = nullptr,
                const GateArgs &ga = GateArgs{}, NodeCols ncl = NodeCols{nullptr}, T *Wout = nullptr) {
    const int64_t ldp = sw.ldp;
    if (!Wout) Wout = sw.W;
    if (sizeof(T) == 8 && v == 2) v = 1;
    if (v < 0 || v >= kShapes || !shape_fits(v, Kp)) fail(L0L2_E_INVALID, "tile shape does not fit the batch");
    dim3 g((unsigned)(pp / kTileTM[v]), (unsigned)(Kp / kTileTN[v]));
    dim3 b((unsigned)(64 * kTileW[v]));
#define L0L2_XTU(PBM, PBN, PW)                                                                                  \
    hipLaunchKernelGGL((k_admm_xtu<T, T, PBM, PBN, PW>), g, b, 0, s, sw.Xh, sw.ldc, sw.U, sw.ldu, np,            \
                       (const T *)sw.W, Wout, sw.beta, sw.V, sw.B, codes, sw.c, active, q, ldp, store_b, gpart, ga, ncl)
#define L0L2_XTUL(WM, WN)                                                                                       \
    hipLaunchKernelGGL((k_admm_xtu_lds<T, WM, WN>), g, b, 0, s, sw.Xh, sw.ldc, sw.U, sw.ldu, np, (const T *)sw.W, \
                       Wout, sw.beta, sw.V, sw.B, codes, sw.c, active, q, ldp, store_b, gpart, ga, ncl)
    if (v >= 9) {
        switch (v) {
            case 9: L0L2_XTUL(2, 2); break;
            case 10: L0L2_XTUL(4, 2); break;
            default: L0L2_XTUL(4, 4); break;
        }
        return;
    }
    switch (v) {
        case 0: L0L2_XTU(2, 2, 4); break;
        case 1: L0L2_XTU(2, 2, 8); break;
        case 2: L0L2_XTU(2, 2, (sizeof(T) == 8 ? 8 : 16)); break;
        case 3: L0L2_XTU(1, 2, 8); break;
        case 4: L0L2_XTU(2, 1, 8); break;
        case 5: L0L2_XTU(1, 1, 4); break;
        case 6: L0L2_XTU(4, 2, 8); break;
        case 7: L0L2_XTU(2, 4, 8); break;
        default: L0L2_XTU(4, 4, 4); break;
    }
#undef L0L2_XTU
#undef L0L2_XTUL
}

// The anchored sweep's contraction over n (FP32 operands, FP64 update).
void launch_xtu_anch(int v, hipStream_t s, const Sweep<float> &s32, const Sweep<double> &s64, const double *Za,
                     const double *Wa, int64_t np, int64_t pp, int64_t Kp, const uint8_t *codes, const int *active,
                     const DevParams<double> &q, int store_b, double *gpart, const GateArgs &ga, NodeCols ncl) {
    if (v < 0 || v >= kShapes || !shape_fits(v, Kp)) fail(L0L2_E_INVALID, "tile shape does not fit the batch");
    dim3 g((unsigned)(pp / kTileTM[v]), (unsigned)(Kp / kTileTN[v]));
    dim3 b((unsigned)(64 * kTileW[v]));
    const int64_t ldp = s32.ldp;
#define L0L2_XTUA(PBM, PBN, PW)                                                                                \
    hipLaunchKernelGGL((k_admm_xtu_anch<PBM, PBN, PW>), g, b, 0, s, s32.Xh, s32.ldc, s32.U, s32.ldu, np, Za, Wa,  \
                       s64.W, s64.beta, s64.V, s64.B, s32.W, codes, s64.c, active, q, ldp, store_b, gpart, ga, ncl)
#define L0L2_XTUAL(WM, WN)                                                                                     \
    hipLaunchKernelGGL((k_admm_xtu_anch_lds<WM, WN>), g, b, 0, s, s32.Xh, s32.ldc, s32.U, s32.ldu, np, Za, Wa,    \
                       s64.W, s64.beta, s64.V, s64.B, s32.W, codes, s64.c, active, q, ldp, store_b, gpart, ga, ncl)
    if (v >= 9) {
        switch (v) {
            case 9: L0L2_XTUAL(2, 2); break;
            case 10: L0L2_XTUAL(4, 2); break;
            default: L0L2_XTUAL(4, 4); break;
        }
        return;
    }
    switch (v) {
        case 0: L0L2_XTUA(2, 2, 4); break;
        case 1: L0L2_XTUA(2, 2, 8); break;
        case 2: L0L2_XTUA(2, 2, 16); break;
        case 3: L0L2_XTUA(1, 2, 8); break;
        case 4: L0L2_XTUA(2, 1, 8); break;
        case 5: L0L2_XTUA(1, 1, 4); break;
        case 6: L0L2_XTUA(4, 2, 8); break;
        case 7: L0L2_XTUA(2, 4, 8); break;
        default: L0L2_XTUA(4, 4, 4); break;
    }
#undef L0L2_XTUA
#undef L0L2_XTUAL
}

// The partial-product buffer of the sliced shapes, sized for kMaxSplit slices of
// the workspace's node capacity (every slot a live column may name; at least Kp)
// with rows of ld elements of elem bytes.  It grows only before a capture (the
// tile choice runs first); a move drops the captured graphs, which hold its
// address.
void ensure_split(l0l2_ctx *ctx, int64_t Kp, int64_t ld, size_t elem) {
    Workspace &ws = ctx->ws;
    const size_t need = (size_t)kMaxSplit * std::max(Kp, ws.cap) * ld * elem;
    if (need <= ws.Upart.bytes) return;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ws.Upart.ensure(need);
    drop_graphs(ctx);
    ++ws.gen;
}
SplitBuf split_buf(l0l2_ctx *ctx) { return SplitBuf{ctx->ws.Upart.ptr, ctx->ws.Upart.bytes, ctx->ws.cap}; }

// Tile shapes chosen for (arithmetic type, padded batch): each shape that fits
// is timed on the live batch (every node masked inactive, so the epilogue
// writes nothing), the best of several interleaved samples per shape, and the
// fastest kept for this instance.
// Shapes without timing (contexts whose timings would vary, such as the
// server's under contention): the LDS-staged 128 x 128 tiles when both
// contractions' grids of them hold at least one workgroup per compute unit,
// else the 32 x 32 register tile (shape 0), whatever the load.
bool big_batch_rule(const Instance &in, int64_t Kp) {
    return Kp % 128 == 0 && (in.np / 128) * (Kp / 128) >= 256 && (in.pp / 128) * (Kp / 128) >= 256;
}

template <class T>
TileChoice &tile_choice(l0l2_ctx *ctx, const Sweep<T> &sw, int64_t Kp) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    ensure_split(ctx, Kp, sw.ldu, sizeof(T));
    if (ctx->force_xw >= 0) {
        static thread_local TileChoice forced;
        forced.xw = ctx->force_xw;
        forced.xtu = ctx->force_xtu;
        return forced;
    }
    const int kind = sizeof(T) == 8 ? 1 : 0;
    auto key = std::make_pair(kind, Kp);
    auto it = in.tiles.find(key);
    if (it != in.tiles.end()) return it->second;
    TileChoice tc;
    if (ctx->tune) {
        hipStream_t s = ctx->stream;
        const int64_t np = in.np, pp = in.pp;
        DevBuf inactive;
        inactive.ensure(sizeof(int) * Kp);
        HIPCHK(hipMemsetAsync(inactive.ptr, 0, sizeof(int) * Kp, s));
        DevParams<T> q = dev_params<T>(in.mp);
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        // time `reps` back-to-back launches of shape v (which = 0: contraction
        // over p, 1: contraction over n with its masked epilogue, 2: the plain
        // product over n that completes an anchor, into the anchor buffer z_a,
        // which every anchored block recomputes before it reads it)
        const bool anchors = sizeof(T) == 8 && in.prec != L0L2_FP64;
        auto time_shape = [&](int v, int which, int reps) {
            HIPCHK(hipEventRecord(e0, s));
            for (int t = 0; t < reps; ++t) {
                if (which == 0)
                    launch_xw<T, T, T>(v, s, sw.XhR, sw.ldr, sw.W, sw.ldp, sw.U, sw.ldu, np, Kp, pp, NodeCols{nullptr},
                                       split_buf(ctx));
                else if (which == 1)
                    launch_xtu<T>(v, s, sw, np, pp, Kp, ws.codes.as<uint8_t>(), inactive.as<int>(), q, 0);
                else
                    launch_xw<T, T, T>(v, s, sw.Xh, sw.ldc, sw.U, sw.ldu, reinterpret_cast<T *>(ws.Za.ptr), sw.ldp, pp,
                                       Kp, np, NodeCols{nullptr});
            }
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            return ms / (float)reps;
        };
        // warm-up round, which also sizes the measurement: about 0.2 ms of work
        // per sample, and fewer rounds for launches longer than 1 ms
        // which = 1 (the contraction over n) has no sliced shapes; a sliced shape
        // is a candidate only where its tile unsliced would leave CUs idle
        // (fewer workgroups than the 256 compute units)
        auto valid = [&](int v, int which) {
            if (!shape_fits(v, Kp)) return false;
            if (which == 2) return anchors && v < kShapes;
            if (v < kShapes) return true;
            return which == 0 && (np / kTileTM[v]) * (Kp / kTileTN[v]) < 256;
        };
        float t0 = 0.f;
        for (int v = 0; v < kShapesXw; ++v)
            for (int which = 0; which < 3; ++which)
                if (valid(v, which)) t0 = std::max(t0, time_shape(v, which, 1));
        const int reps = std::max(1, std::min(8, (int)(0.2f / std::max(t0, 1e-4f))));
        const int rounds = t0 > 1.0f ? 2 : 4;
        float best[kShapesXw][3];
        for (int v = 0; v < kShapesXw; ++v) best[v][0] = best[v][1] = best[v][2] = 1e30f;
        for (int r = 0; r < rounds; ++r)
            for (int v = 0; v < kShapesXw; ++v)
                for (int which = 0; which < 3; ++which)
                    if (valid(v, which)) best[v][which] = std::min(best[v][which], time_shape(v, which, reps));
        float best_xw = 1e30f, best_xtu = 1e30f, best_z2 = 1e30f;
        for (int v = 0; v < kShapesXw; ++v) {
            if (valid(v, 0) && best[v][0] < best_xw) { best_xw = best[v][0]; tc.xw = v; }
            if (valid(v, 1) && best[v][1] < best_xtu) { best_xtu = best[v][1]; tc.xtu = v; }
            if (valid(v, 2) && best[v][2] < best_z2) { best_z2 = best[v][2]; tc.z2 = v; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIPCHK(hipGetLastError());
    }
    if (!ctx->tune && big_batch_rule(in, Kp)) tc.xw = tc.xtu = 11;   // LDS-staged 128 x 128
    return in.tiles[key] = tc;
}

// ---------------------------------------------------------------------------
// Host drivers
// ---------------------------------------------------------------------------
// The active list of the current batch.
NodeCols active_cols(l0l2_ctx *ctx) { return NodeCols{ctx->ws.list.as<int>()}; }

GateArgs gate_args(const Instance &in) {
    GateArgs g;
    g.l0 = in.mp.l0; g.l2 = in.mp.l2; g.M = in.mp.M; g.s = in.mp.s;
    g.two_M_l2 = in.mp.two_M_l2; g.four_l2 = in.mp.four_l2; g.l2_M2 = in.mp.l2_M2; g.psi_lin = in.mp.psi_lin;
    g.free_quad = in.mp.free_quad;
    return g;
}

// One sweep; with gate set the epilogue also leaves the per-tile sums of the
// gap estimate in ws.gpart.
template <class T>
void sweep_once(l0l2_ctx *ctx, const Sweep<T> &sw, int64_t Kp, bool store_b, int64_t active, bool gate = false) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    const int64_t np = in.np, pp = in.pp;
    DevParams<T> q = dev_params<T>(in.mp);
    const TileChoice &tc = tile_choice<T>(ctx, sw, Kp);
    prof_begin(ctx, prof_xw<T>());
    launch_xw<T, T, T>(tc.xw, s, sw.XhR, sw.ldr, sw.W, sw.ldp, sw.U, sw.ldu, np, Kp, pp, active_cols(ctx),
                       split_buf(ctx));
    prof_end(ctx, prof_xw<T>(), active);
    prof_begin(ctx, prof_xtu<T>());
    launch_xtu<T>(tc.xtu, s, sw, np, pp, Kp, ws.codes.as<uint8_t>(), ws.active.as<int>(), q, store_b ? 1 : 0,
                  gate ? ws.gpart.as<double>() : nullptr, gate_args(in), active_cols(ctx));
    prof_end(ctx, prof_xtu<T>(), active);
    HIPCHK(hipGetLastError());
}

// Tile shapes of the BF16 split form: 0 = register tile 32 x 32 (8 waves split
// the contraction), 1 = LDS-staged 64 x 64, 2 = LDS-staged 128 x 128.
// 3, 4 (contraction over p only): the register tile with the range cut into 4
// or 8 slices.
constexpr int kShapesBf16 = 3, kShapesBf16Xw = 7;
constexpr int kBfTM[kShapesBf16Xw] = {32, 64, 128, 32, 32, 128, 128};
constexpr int kBfTN[kShapesBf16Xw] = {32, 64, 128, 32, 32, 128, 128};
constexpr int kBfSplit[kShapesBf16Xw] = {1, 1, 1, 4, 8, 4, 8};

void launch_xw_bf16(int v, l0l2_ctx *ctx, const float *B, float *U, int64_t Kp, NodeCols ncl) {
    Instance &in = ctx->inst;
    const int64_t np = in.np, pp = in.pp;
    if (v < 0 || v >= kShapesBf16Xw || Kp % kBfTN[v] != 0) fail(L0L2_E_INVALID, "tile shape does not fit the batch");
    dim3 g((unsigned)(np / kBfTM[v]), (unsigned)(Kp / kBfTN[v]));
    const __bf16 *hi = in.XhR.as<__bf16>(), *lo = in.XhRLo.as<__bf16>();
    const int64_t lda = in.ldwr, ldb = in.ldp, ldu = in.ldu;
    if (v >= kShapesBf16) {
        // no slice may be empty: at most one per 32-wide chunk (LDS) or 64-wide pair (register)
        const int S = (int)std::min<int64_t>(kBfSplit[v], v >= 5 ? pp / 32 : pp / 64);
        SplitBuf sk = split_buf(ctx);
        const int64_t pstride = sk.rows * ldu;
        if (sk.rows < Kp || (size_t)S * pstride * sizeof(float) > sk.bytes)
            fail(L0L2_E_INVALID, "split buffer too small");
        float *P = static_cast<float *>(sk.ptr);
        if (v >= 5)
            hipLaunchKernelGGL((k_gemm_xw_bf16_lds<4, 4>), dim3(g.x, g.y, (unsigned)S), dim3(256), 0, ctx->stream, hi,
                               lo, lda, B, ldb, P, ldu, pp, ncl, pstride);
        else
            hipLaunchKernelGGL(k_gemm_xw_bf16, dim3(g.x, g.y, (unsigned)S), dim3(64 * kWavesBf16), 0, ctx->stream, hi,
                               lo, lda, B, ldb, P, ldu, pp, ncl, pstride);
        hipLaunchKernelGGL(k_splitk_sum<float>, dim3((unsigned)((np + 255) / 256), (unsigned)Kp), dim3(256), 0,
                           ctx->stream, (const float *)P, pstride, S, U, ldu, np, ncl);
        return;
    }
    if (v == 0)
        hipLaunchKernelGGL(k_gemm_xw_bf16, g, dim3(64 * kWavesBf16), 0, ctx->stream, hi, lo, lda, B, ldb, U, ldu, pp,
                           ncl, (int64_t)0);
    else if (v == 1)
        hipLaunchKernelGGL((k_gemm_xw_bf16_lds<2, 2>), g, dim3(256), 0, ctx->stream, hi, lo, lda, B, ldb, U, ldu, pp,
                           ncl, (int64_t)0);
    else
        hipLaunchKernelGGL((k_gemm_xw_bf16_lds<4, 4>), g, dim3(256), 0, ctx->stream, hi, lo, lda, B, ldb, U, ldu, pp,
                           ncl, (int64_t)0);
}

// Operands of a Gram-form sweep in the BF16 split form: G's BF16 pair over the
// range p, the node operand (W, or d when anchored) read from win, the new W
// (or d) written to wout.
struct GramBf {
    const __bf16 *hi, *lo;
    int64_t lda;
    float *win, *wout;
};

// Contraction over n in the BF16 split form (over p with G when gr is given):
// FP32 update (anch = false, on the FP32 state) or the anchored FP64 update
// (anch = true).
void launch_xtu_bf16(int v, l0l2_ctx *ctx, bool anch, int64_t Kp, const int *active, int store_b, double *gpart,
                     NodeCols ncl, const GramBf *gr = nullptr) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    const int64_t pp = in.pp;
    if (v < 0 || v >= kShapesBf16 || Kp % kBfTN[v] != 0) fail(L0L2_E_INVALID, "tile shape does not fit the batch");
    dim3 g((unsigned)(pp / kBfTM[v]), (unsigned)(Kp / kBfTN[v]));
    Sweep<float> s32 = sweep32(ctx);
    const __bf16 *hi = gr ? gr->hi : in.Xh.as<__bf16>(), *lo = gr ? gr->lo : in.XhLo.as<__bf16>();
    const int64_t lda = gr ? gr->lda : in.ldw, ldu = gr ? in.ldp : in.ldu, ldp = in.ldp;
    const int64_t np = gr ? pp : in.np;   // the contraction's range
    const float *U = gr ? gr->win : s32.U;
    const float *wr = gr ? gr->win : s32.W;
    float *ww = gr ? gr->wout : s32.W;
    Sweep<double> s64 = sweep64(ctx);
    const DevParams<float> q32 = dev_params<float>(in.mp);
    const DevParams<double> q64 = dev_params<double>(in.mp);
    const GateArgs ga = gate_args(in);
    const double *Za = ws.Za.as<double>(), *Wa = ws.Wa.as<double>();
    const uint8_t *codes = ws.codes.as<uint8_t>();
    hipStream_t s = ctx->stream;
    if (v == 0) {
        if (anch)
            hipLaunchKernelGGL(k_admm_xtu_anch_bf16, g, dim3(64 * kWavesBf16), 0, s, hi, lo, lda, U, ldu, np, Za,
                               Wa, s64.W, s64.beta, s64.V, s64.B, ww, codes, s64.c, active, q64, ldp, store_b,
                               gpart, ga, ncl);
        else
            hipLaunchKernelGGL(k_admm_xtu_bf16, g, dim3(64 * kWavesBf16), 0, s, hi, lo, lda, U, ldu, np, wr, ww,
                               s32.beta, s32.V, s32.B, codes, s32.c, active, q32, ldp, store_b, gpart, ga, ncl);
        return;
    }
#define L0L2_XTUB(WM, WN, A)                                                                                    \
    hipLaunchKernelGGL((k_admm_xtu_bf16_lds<WM, WN, A>), g, dim3(256), 0, s, hi, lo, lda, U, ldu, np, wr, ww,     \
                       s32.beta, s32.V, s32.B, Za, Wa, s64.W, s64.beta, s64.V, s64.B, codes, s32.c, s64.c, active, \
                       q32, q64, ldp, store_b, gpart, ga, ncl)
    if (v == 1) {
        if (anch) L0L2_XTUB(2, 2, 1);
        else L0L2_XTUB(2, 2, 0);
    } else {
        if (anch) L0L2_XTUB(4, 4, 1);
        else L0L2_XTUB(4, 4, 0);
    }
#undef L0L2_XTUB
}

// BF16 shapes chosen per padded batch, timed like tile_choice (kind 2).
TileChoice &tile_choice_bf16(l0l2_ctx *ctx, int64_t Kp) {
    Instance &in = ctx->inst;
    ensure_split(ctx, Kp, in.ldu, sizeof(float));
    if (ctx->force_xw >= 0) {
        // fixed shapes: 0-11 map to the three unsliced shapes; the sliced ones to
        // the register tile in 4 slices (14, 16) or 8 (15), the 128 x 128
        // LDS-staged tile in 4 slices (12, 13) or 8 (17)
        static thread_local TileChoice forced;
        const int f = ctx->force_xw;
        forced.xw = f < kShapes ? std::min(f, kShapesBf16 - 1) : f == 15 ? 4 : (f == 12 || f == 13) ? 5 : f == 17 ? 6 : 3;
        forced.xtu = std::min(ctx->force_xtu, kShapesBf16 - 1);
        return forced;
    }
    auto key = std::make_pair(2, Kp);
    auto it = in.tiles.find(key);
    if (it != in.tiles.end()) return it->second;
    TileChoice tc;
    tc.xw = tc.xtu = 0;
    if (ctx->tune) {
        hipStream_t s = ctx->stream;
        DevBuf inactive;
        inactive.ensure(sizeof(int) * Kp);
        HIPCHK(hipMemsetAsync(inactive.ptr, 0, sizeof(int) * Kp, s));
        Sweep<float> s32 = sweep32(ctx);
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        auto time_shape = [&](int v, int which, int reps) {
            HIPCHK(hipEventRecord(e0, s));
            for (int t = 0; t < reps; ++t) {
                if (which == 0) launch_xw_bf16(v, ctx, s32.W, s32.U, Kp, NodeCols{nullptr});
                else launch_xtu_bf16(v, ctx, false, Kp, inactive.as<int>(), 0, nullptr, NodeCols{nullptr});
            }
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            return ms / (float)reps;
        };
        // sliced shapes: the contraction over p only, where the unsliced grid
        // would leave compute units idle
        auto valid = [&](int v, int which) {
            if (Kp % kBfTN[v] != 0) return false;
            if (v < kShapesBf16) return true;
            return which == 0 && (in.np / kBfTM[v]) * (Kp / kBfTN[v]) < 256;
        };
        float t0 = 0.f;
        for (int v = 0; v < kShapesBf16Xw; ++v)
            for (int which = 0; which < 2; ++which)
                if (valid(v, which)) t0 = std::max(t0, time_shape(v, which, 1));
        const int reps = std::max(1, std::min(8, (int)(0.2f / std::max(t0, 1e-4f))));
        const int rounds = t0 > 1.0f ? 2 : 4;
        float best[kShapesBf16Xw][2];
        for (int v = 0; v < kShapesBf16Xw; ++v) best[v][0] = best[v][1] = 1e30f;
        for (int r = 0; r < rounds; ++r)
            for (int v = 0; v < kShapesBf16Xw; ++v)
                for (int which = 0; which < 2; ++which)
                    if (valid(v, which)) best[v][which] = std::min(best[v][which], time_shape(v, which, reps));
        float bx = 1e30f, bt = 1e30f;
        for (int v = 0; v < kShapesBf16Xw; ++v) {
            if (valid(v, 0) && best[v][0] < bx) { bx = best[v][0]; tc.xw = v; }
            if (valid(v, 1) && best[v][1] < bt) { bt = best[v][1]; tc.xtu = v; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIPCHK(hipGetLastError());
    }
    if (!ctx->tune && big_batch_rule(in, Kp)) tc.xw = tc.xtu = 2;    // LDS-staged 128 x 128
    return in.tiles[key] = tc;
}

// One sweep of the BF16 form on the FP32 state (anch = false), or an anchored
// sweep in BF16 mode (anch = true: products of d = W - w_a, FP64 update).
void sweep_once_bf16(l0l2_ctx *ctx, int64_t Kp, bool store_b, int64_t active, bool gate, bool anch) {
    Workspace &ws = ctx->ws;
    Sweep<float> s32 = sweep32(ctx);
    const TileChoice &tc = tile_choice_bf16(ctx, Kp);
    prof_begin(ctx, PROF_GEMM_XW_BF16);
    launch_xw_bf16(tc.xw, ctx, s32.W, s32.U, Kp, active_cols(ctx));
    prof_end(ctx, PROF_GEMM_XW_BF16, active);
    prof_begin(ctx, PROF_ADMM_XTU_BF16);
    launch_xtu_bf16(tc.xtu, ctx, anch, Kp, ws.active.as<int>(), store_b ? 1 : 0, gate ? ws.gpart.as<double>() : nullptr,
                    active_cols(ctx));
    prof_end(ctx, PROF_ADMM_XTU_BF16, active);
    HIPCHK(hipGetLastError());
}

// Start of an anchored block: w_a = W (FP64), d = 0, z_a = Xh^T (Xh w_a) in FP64.
void anchor_start(l0l2_ctx *ctx, int64_t Kp, int64_t cols) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    const int64_t np = in.np, pp = in.pp;
    Sweep<double> s64 = sweep64(ctx);
    Sweep<float> s32 = sweep32(ctx);
    const TileChoice &tc = tile_choice<double>(ctx, s64, cols);
    prof_begin(ctx, PROF_ANCHOR);
    const int64_t ldp = in.ldp;
    hipLaunchKernelGGL(k_anchor_init, dim3(grid1d(Kp * ldp)), dim3(256), 0, s, s64.W, ws.Wa.as<double>(), s32.W,
                       Kp * ldp);
    launch_xw<double, double, double>(tc.xw, s, s64.XhR, s64.ldr, ws.Wa.as<double>(), ldp, s64.U, s64.ldu, np, cols,
                                      pp, active_cols(ctx), split_buf(ctx));
    // the second product runs over n (short) into a p x nodes output: its own
    // timed shape, else (fixed shapes) the contraction over p's unless that is
    // sliced, then the contraction over n's
    const int v2 = tc.z2 >= 0 ? tc.z2 : (split_of(tc.xw) > 1 ? tc.xtu : tc.xw);
    launch_xw<double, double, double>(v2, s, s64.Xh, s64.ldc, s64.U, s64.ldu, ws.Za.as<double>(), ldp, pp, cols,
                                      np, active_cols(ctx));
    prof_end(ctx, PROF_ANCHOR);
    HIPCHK(hipGetLastError());
}

// One anchored sweep: U = Xh d (FP32), then the FP64 update from z_a + Xh^T U.
void sweep_once_anch(l0l2_ctx *ctx, int64_t Kp, bool store_b, int64_t active, bool gate) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    const int64_t np = in.np, pp = in.pp;
    Sweep<float> s32 = sweep32(ctx);
    Sweep<double> s64 = sweep64(ctx);
    const TileChoice &tc = tile_choice<float>(ctx, s32, Kp);
    prof_begin(ctx, PROF_GEMM_XW_F32);
    launch_xw<float, float, float>(tc.xw, s, s32.XhR, s32.ldr, s32.W, s32.ldp, s32.U, s32.ldu, np, Kp, pp,
                                   active_cols(ctx), split_buf(ctx));
    prof_end(ctx, PROF_GEMM_XW_F32, active);
    prof_begin(ctx, PROF_ADMM_XTU_F32);
    launch_xtu_anch(tc.xtu, s, s32, s64, ws.Za.as<double>(), ws.Wa.as<double>(), np, pp, Kp,
                    ws.codes.as<uint8_t>(), ws.active.as<int>(), dev_params<double>(in.mp), store_b ? 1 : 0,
                    gate ? ws.gpart.as<double>() : nullptr, gate_args(in), active_cols(ctx));
    prof_end(ctx, PROF_ADMM_XTU_F32, active);
    HIPCHK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Gram form of the b-update (FP32 mode).  With G = Xh^T Xh (p x p, symmetric;
// Xh = L^{-1} X), b = D w = (w - G w) / rho: one contraction over p per sweep
// instead of two (over p, then over n), the paper's p x p form of D written
// through the folded operand.  Its work per node-sweep is 2 p^2 against 4 n p,
// and it halves the launches per sweep, so it is taken when p <= 1.5 n (and G
// stays small).  The contraction's node operand is W itself, which the same
// launch updates, so W alternates between two buffers (the anchored sweeps: d).
// ---------------------------------------------------------------------------
__global__ void k_f64_to_f32(const double *__restrict__ src, int64_t lds, float *__restrict__ dst, int64_t ldd,
                             int64_t rows, int64_t cols) {
    const int64_t r = blockIdx.y, j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < rows && j < cols) dst[r * ldd + j] = (float)src[r * lds + j];
}

__global__ void k_f64_to_bf16x2(const double *__restrict__ src, int64_t lds, __bf16 *__restrict__ hi,
                                __bf16 *__restrict__ lo, int64_t ldd, int64_t rows, int64_t cols) {
    const int64_t r = blockIdx.y, j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < rows && j < cols) {
        const float x = (float)src[r * lds + j];
        const __bf16 h = (__bf16)x;
        hi[r * ldd + j] = h;
        lo[r * ldd + j] = (__bf16)(x - (float)h);
    }
}

// The Gram form is a candidate in FP32 and BF16 modes when its contraction
// (2 p^2 flops per node-sweep) can beat the folded form's two (4 n p), i.e.
// p < 2 n, and G (padded p squared in FP64 plus its working copies) stays
// within padded p <= 8192.  Among candidates the form is measured on the first
// solve (decide_form); before that, and where it is not measured, the Gram form
// is assumed when p <= 1.5 n.
bool gram_candidate(const Instance &in) {
    return (in.prec == L0L2_FP32 || in.prec == L0L2_BF16) && in.pp <= 2 * in.np && in.pp <= 8192;
}

bool gram_form(const l0l2_ctx *ctx) {
    const Instance &in = ctx->inst;
    if ((in.prec != L0L2_FP32 && in.prec != L0L2_BF16) || ctx->bform == 1) return false;
    if (ctx->bform == 2) return true;
    if (!gram_candidate(in)) return false;
    if (in.form_pick) return in.form_pick == 2;
    return 2 * in.pp <= 3 * in.np;
}

// G in FP64 (the anchors) and FP32 (the sweeps), once per instance.
void ensure_gram(l0l2_ctx *ctx) {
    Instance &in = ctx->inst;
    if (in.gram_built) return;
    hipStream_t s = ctx->stream;
    const int64_t pp = in.pp, np = in.np;
    in.ldg64 = ld_pad(pp, 8);
    in.ldg32 = ld_pad(pp, 4);
    in.G64.ensure(sizeof(double) * pp * in.ldg64);
    in.G32.ensure(sizeof(float) * pp * in.ldg32);
    // G[j][i] = sum_r Xh[r][i] Xh[r][j]: rows of the column-major Xh64 are columns of Xh
    launch_xw<double, double, double>(0, s, in.Xh64.as<double>(), in.ldx, in.Xh64.as<double>(), in.ldx,
                                      in.G64.as<double>(), in.ldg64, pp, pp, np);
    hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)((pp + 255) / 256), (unsigned)pp), dim3(256), 0, s,
                       in.G64.as<double>(), in.ldg64, in.G32.as<float>(), in.ldg32, pp, pp);
    if (in.prec == L0L2_BF16) {
        in.ldgb = ld_pad(pp, 2);
        in.Ghi.ensure(sizeof(__bf16) * pp * in.ldgb);
        in.Glo.ensure(sizeof(__bf16) * pp * in.ldgb);
        hipLaunchKernelGGL(k_f64_to_bf16x2, dim3((unsigned)((pp + 255) / 256), (unsigned)pp), dim3(256), 0, s,
                           in.G64.as<double>(), in.ldg64, in.Ghi.as<__bf16>(), in.Glo.as<__bf16>(), in.ldgb, pp, pp);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    in.gram_built = true;
}

// Sweep t (1-based) of a block reads the W (or d) buffer it names and writes the
// other: odd sweeps ws.W -> ws.W2, even ones back.
float *gram_in(l0l2_ctx *ctx, int t) { return (t & 1) ? ctx->ws.W.as<float>() : ctx->ws.W2.as<float>(); }
float *gram_out(l0l2_ctx *ctx, int t) { return (t & 1) ? ctx->ws.W2.as<float>() : ctx->ws.W.as<float>(); }

// One Gram-form sweep on the FP32 state.
void sweep_once_gram(l0l2_ctx *ctx, int64_t Kp, bool store_b, int64_t active, bool gate, int t) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    Sweep<float> s32 = sweep32(ctx);
    const TileChoice &tc = tile_choice<float>(ctx, s32, Kp);
    Sweep<float> g = s32;
    g.Xh = in.G32.as<float>();
    g.ldc = in.ldg32;
    g.W = gram_in(ctx, t);
    g.U = g.W;
    g.ldu = in.ldp;
    prof_begin(ctx, PROF_ADMM_XTU_F32);
    launch_xtu<float>(tc.xtu, ctx->stream, g, in.pp, in.pp, Kp, ws.codes.as<uint8_t>(), ws.active.as<int>(),
                      dev_params<float>(in.mp), store_b ? 1 : 0, gate ? ws.gpart.as<double>() : nullptr,
                      gate_args(in), active_cols(ctx), gram_out(ctx, t));
    prof_end(ctx, PROF_ADMM_XTU_F32, active);
    HIPCHK(hipGetLastError());
}

bool bf16_single(l0l2_ctx *ctx, int64_t cols);
__bf16 *dbf_in(l0l2_ctx *ctx, int t);

// Start of an anchored Gram-form block: w_a = W (FP64), d = 0 (in ws.W, or in
// the BF16 operand of single-term sweeps), z_a = G w_a.
void anchor_start_gram(l0l2_ctx *ctx, int64_t Kp, int64_t cols) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    Sweep<double> s64 = sweep64(ctx);
    Sweep<float> s32 = sweep32(ctx);
    const TileChoice &tc = tile_choice<double>(ctx, s64, cols);
    prof_begin(ctx, PROF_ANCHOR);
    const int64_t ldp = in.ldp;
    if (bf16_single(ctx, cols))
        hipLaunchKernelGGL(k_anchor_init_bf, dim3(grid1d(Kp * ldp)), dim3(256), 0, s, s64.W, ws.Wa.as<double>(),
                           dbf_in(ctx, 1), Kp * ldp);
    else
        hipLaunchKernelGGL(k_anchor_init, dim3(grid1d(Kp * ldp)), dim3(256), 0, s, s64.W, ws.Wa.as<double>(), s32.W,
                           Kp * ldp);
    const int v = tc.z2 >= 0 ? tc.z2 : (split_of(tc.xw) > 1 ? tc.xtu : tc.xw);
    launch_xw<double, double, double>(v, s, in.G64.as<double>(), in.ldg64, ws.Wa.as<double>(), ldp,
                                      ws.Za.as<double>(), ldp, in.pp, cols, in.pp, active_cols(ctx));
    prof_end(ctx, PROF_ANCHOR);
    HIPCHK(hipGetLastError());
}

// One anchored Gram-form sweep: Q = z_a + G32 d_in, FP64 update, d_out = fl32(W - w_a).
void sweep_once_anch_gram(l0l2_ctx *ctx, int64_t Kp, bool store_b, int64_t active, bool gate, int t) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    Sweep<float> s32 = sweep32(ctx);
    Sweep<double> s64 = sweep64(ctx);
    const TileChoice &tc = tile_choice<float>(ctx, s32, Kp);
    Sweep<float> g = s32;
    g.Xh = in.G32.as<float>();
    g.ldc = in.ldg32;
    g.U = gram_in(ctx, t);
    g.ldu = in.ldp;
    g.W = gram_out(ctx, t);   // the d the update writes
    prof_begin(ctx, PROF_ADMM_XTU_F32);
    launch_xtu_anch(tc.xtu, ctx->stream, g, s64, ws.Za.as<double>(), ws.Wa.as<double>(), in.pp, in.pp, Kp,
                    ws.codes.as<uint8_t>(), ws.active.as<int>(), dev_params<double>(in.mp), store_b ? 1 : 0,
                    gate ? ws.gpart.as<double>() : nullptr, gate_args(in), active_cols(ctx));
    prof_end(ctx, PROF_ADMM_XTU_F32, active);
    HIPCHK(hipGetLastError());
}

// Single-term BF16 blocks of the Gram form (the default where the LDS-staged
// tiles are chosen): each block is anchored and its sweeps multiply only the
// movement d since the anchor, with one BF16 term of G and of d (one MFMA per
// product instead of the split form's three).  FP32 phase: the block's first
// sweep is a split-form sweep whose product and operand become the FP32 anchor;
// FP64 phase: the FP64 anchor of anchor_start_gram.  Operand d alternates
// between two BF16 buffers: sweep t reads Dbf[t & 1] and writes Dbf[(t + 1) & 1].
bool bf16_single(l0l2_ctx *ctx, int64_t cols) {
    const Instance &in = ctx->inst;
    return in.prec == L0L2_BF16 && ctx->bf16_terms == 1 && gram_form(ctx) && tile_choice_bf16(ctx, cols).xtu >= 1;
}

__bf16 *dbf_in(l0l2_ctx *ctx, int t) { return ctx->ws.Dbf[t & 1].as<__bf16>(); }
__bf16 *dbf_out(l0l2_ctx *ctx, int t) { return ctx->ws.Dbf[(t + 1) & 1].as<__bf16>(); }

// mode 1: FP32 state and anchor; mode 2: FP64 state and anchor.
void launch_xtu_bf16s(int v, l0l2_ctx *ctx, int mode, int64_t Kp, int store_b, double *gpart, NodeCols ncl, int t) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    if (v < 1 || v >= kShapesBf16 || Kp % kBfTN[v] != 0) fail(L0L2_E_INVALID, "tile shape does not fit the batch");
    dim3 g((unsigned)(in.pp / kBfTM[v]), (unsigned)(Kp / kBfTN[v]));
    Sweep<float> s32 = sweep32(ctx);
    Sweep<double> s64 = sweep64(ctx);
    const DevParams<float> q32 = dev_params<float>(in.mp);
    const DevParams<double> q64 = dev_params<double>(in.mp);
    const GateArgs ga = gate_args(in);
    const __bf16 *A = in.Ghi.as<__bf16>();
    const float *wr = gram_in(ctx, t);
    float *ww = gram_out(ctx, t);
#define L0L2_XTUS(WM, WN, MODE)                                                                                    \
    hipLaunchKernelGGL((k_admm_xtu_bf16s_lds<WM, WN, MODE>), g, dim3(256), 0, ctx->stream, A, in.ldgb,             \
                       (const __bf16 *)dbf_in(ctx, t), dbf_out(ctx, t), in.pp, wr, ww, s32.beta, s32.V, s32.B,     \
                       ws.Za32.as<float>(), ws.Wa32.as<float>(), ws.Za.as<double>(), ws.Wa.as<double>(), s64.W,   \
                       s64.beta, s64.V, s64.B, ws.codes.as<uint8_t>(), s32.c, s64.c, ws.active.as<int>(), q32,   \
                       q64, in.ldp, store_b, gpart, ga, ncl)
    if (v == 1) {
        if (mode == 2) L0L2_XTUS(2, 2, 2);
        else L0L2_XTUS(2, 2, 1);
    } else if (ctx->bf16_rows == 256 && in.pp % 256 == 0) {
        // 256 x 128 tile: the grid's rows halve (the estimate stays per 128 rows)
        g.x = (unsigned)(in.pp / 256);
        if (mode == 2) L0L2_XTUS(8, 4, 2);
        else L0L2_XTUS(8, 4, 1);
    } else {
        if (mode == 2) L0L2_XTUS(4, 4, 2);
        else L0L2_XTUS(4, 4, 1);
    }
#undef L0L2_XTUS
}

// The first sweep of an FP32-phase single-term block: a split-form sweep that
// also writes the block's FP32 anchor (z = G w in Za32, w in Wa32) and d.
void launch_xtu_bf16_start(int v, l0l2_ctx *ctx, int64_t Kp, int store_b, double *gpart, NodeCols ncl, int t) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    if (v < 1 || v >= kShapesBf16 || Kp % kBfTN[v] != 0) fail(L0L2_E_INVALID, "tile shape does not fit the batch");
    dim3 g((unsigned)(in.pp / kBfTM[v]), (unsigned)(Kp / kBfTN[v]));
    Sweep<float> s32 = sweep32(ctx);
    Sweep<double> s64 = sweep64(ctx);
    const DevParams<float> q32 = dev_params<float>(in.mp);
    const DevParams<double> q64 = dev_params<double>(in.mp);
    const GateArgs ga = gate_args(in);
    const float *wr = gram_in(ctx, t);
    float *ww = gram_out(ctx, t);
#define L0L2_XTUA(WM, WN)                                                                                          \
    hipLaunchKernelGGL((k_admm_xtu_bf16_lds<WM, WN, 2>), g, dim3(256), 0, ctx->stream, in.Ghi.as<__bf16>(),        \
                       in.Glo.as<__bf16>(), in.ldgb, wr, in.ldp, in.pp, wr, ww, s32.beta, s32.V, s32.B,           \
                       ws.Za.as<double>(), ws.Wa.as<double>(), s64.W, s64.beta, s64.V, s64.B,                     \
                       ws.codes.as<uint8_t>(), s32.c, s64.c, ws.active.as<int>(), q32, q64, in.ldp, store_b,      \
                       gpart, ga, ncl, ws.Za32.as<float>(), ws.Wa32.as<float>(), dbf_out(ctx, t))
    if (v == 1) L0L2_XTUA(2, 2);
    else L0L2_XTUA(4, 4);
#undef L0L2_XTUA
}

// One Gram-form sweep in BF16 mode (anch: the anchored FP64 update).  Split form
// in every sweep, or single-term blocks (bf16_single).
void sweep_once_bf16_gram(l0l2_ctx *ctx, int64_t Kp, bool store_b, int64_t active, bool gate, bool anch, int t) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    const TileChoice &tc = tile_choice_bf16(ctx, Kp);
    double *gp = gate ? ws.gpart.as<double>() : nullptr;
    prof_begin(ctx, PROF_ADMM_XTU_BF16);
    if (bf16_single(ctx, Kp)) {
        if (anch) launch_xtu_bf16s(tc.xtu, ctx, 2, Kp, store_b ? 1 : 0, gp, active_cols(ctx), t);
        else if (t == 1) launch_xtu_bf16_start(tc.xtu, ctx, Kp, store_b ? 1 : 0, gp, active_cols(ctx), t);
        else launch_xtu_bf16s(tc.xtu, ctx, 1, Kp, store_b ? 1 : 0, gp, active_cols(ctx), t);
    } else {
        const GramBf gr{in.Ghi.as<__bf16>(), in.Glo.as<__bf16>(), in.ldgb, gram_in(ctx, t), gram_out(ctx, t)};
        launch_xtu_bf16(tc.xtu, ctx, anch, Kp, ws.active.as<int>(), store_b ? 1 : 0, gp, active_cols(ctx), &gr);
    }
    prof_end(ctx, PROF_ADMM_XTU_BF16, active);
    HIPCHK(hipGetLastError());
}

// Contraction over n of the FP8 form: shape 0 = register tile 32 x 32 (8
// waves), 1 = LDS-staged 64 x 64, 2 = LDS-staged 128 x 128.
constexpr int kShapesFp8 = 3;
constexpr int kF8TM[kShapesFp8] = {32, 64, 128};
constexpr int kF8TN[kShapesFp8] = {32, 64, 128};

void launch_xtu_fp8(int v, l0l2_ctx *ctx, int64_t Kp, const int *active, int store_b, double *gpart, NodeCols ncl) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    if (v < 0 || v >= kShapesFp8 || Kp % kF8TN[v] != 0) fail(L0L2_E_INVALID, "tile shape does not fit the batch");
    Sweep<float> s32 = sweep32(ctx);
    Sweep<double> s64 = sweep64(ctx);
    dim3 g((unsigned)(in.pp / kF8TM[v]), (unsigned)(Kp / kF8TN[v]));
#define L0L2_XTUF8(KER, NT)                                                                                     \
    hipLaunchKernelGGL(KER, g, dim3(NT), 0, ctx->stream, in.qC.as<uint8_t>(), in.ldqc, in.qs.as<float>(), s32.U,   \
                       in.ldu, in.np, ws.Za.as<double>(), ws.Wa.as<double>(), s64.W, s64.beta, s64.V, s64.B, s32.W, \
                       ws.codes.as<uint8_t>(), s64.c, active, dev_params<double>(in.mp), in.ldp, store_b, gpart,    \
                       gate_args(in), ncl)
    if (v == 0) L0L2_XTUF8(k_admm_xtu_fp8, 64 * kWavesBf16);
    else if (v == 1) L0L2_XTUF8((k_admm_xtu_fp8_lds<2, 2>), 256);
    else L0L2_XTUF8((k_admm_xtu_fp8_lds<4, 4>), 256);
#undef L0L2_XTUF8
}

// Contraction over p in FP8 storage: 0-2 = the 32 x 32 register tile (8 waves)
// unsliced or in 4 / 8 slices; 3, 4 = the 128 x 128 LDS-staged tile in 4 / 8
// slices.
constexpr int kShapesFp8Xw = 5;
constexpr int kFp8XwSplit[kShapesFp8Xw] = {1, 4, 8, 4, 8};
constexpr int kF8XwT[kShapesFp8Xw] = {32, 32, 32, 128, 128};

void launch_xw_fp8(int v, l0l2_ctx *ctx, const float *B, float *U, int64_t Kp, NodeCols ncl) {
    Instance &in = ctx->inst;
    if (v < 0 || v >= kShapesFp8Xw || Kp % kF8XwT[v] != 0) fail(L0L2_E_INVALID, "tile shape does not fit the batch");
    if (v >= 3) {
        // no slice may be empty: at most one per 32-wide chunk
        const int S = (int)std::min<int64_t>(kFp8XwSplit[v], in.pp / 32);
        SplitBuf sk = split_buf(ctx);
        const int64_t pstride = sk.rows * in.ldu;
        if (sk.rows < Kp || (size_t)S * pstride * sizeof(float) > sk.bytes)
            fail(L0L2_E_INVALID, "split buffer too small");
        float *P = static_cast<float *>(sk.ptr);
        hipLaunchKernelGGL((k_gemm_xw_fp8_lds<4, 4>), dim3((unsigned)(in.np / 128), (unsigned)(Kp / 128), (unsigned)S),
                           dim3(256), 0, ctx->stream, in.qR.as<uint8_t>(), in.ldqr, in.qs.as<float>(), B, in.ldp, P,
                           in.ldu, in.pp, ncl, pstride);
        hipLaunchKernelGGL(k_splitk_sum<float>, dim3((unsigned)((in.np + 255) / 256), (unsigned)Kp), dim3(256), 0,
                           ctx->stream, (const float *)P, pstride, S, U, in.ldu, in.np, ncl);
        return;
    }
    const int S = (int)std::min<int64_t>(kFp8XwSplit[v], in.pp / 64);
    const dim3 g((unsigned)(in.np / 32), (unsigned)(Kp / 32), (unsigned)S), b(64 * kWavesBf16);
    if (S == 1) {
        hipLaunchKernelGGL(k_gemm_xw_fp8, g, b, 0, ctx->stream, in.qR.as<uint8_t>(), in.ldqr, in.qs.as<float>(), B,
                           in.ldp, U, in.ldu, in.pp, ncl, (int64_t)0);
        return;
    }
    SplitBuf sk = split_buf(ctx);
    const int64_t pstride = sk.rows * in.ldu;
    if (sk.rows < Kp || (size_t)S * pstride * sizeof(float) > sk.bytes) fail(L0L2_E_INVALID, "split buffer too small");
    float *P = static_cast<float *>(sk.ptr);
    hipLaunchKernelGGL(k_gemm_xw_fp8, g, b, 0, ctx->stream, in.qR.as<uint8_t>(), in.ldqr, in.qs.as<float>(), B,
                       in.ldp, P, in.ldu, in.pp, ncl, pstride);
    hipLaunchKernelGGL(k_splitk_sum<float>, dim3((unsigned)((in.np + 255) / 256), (unsigned)Kp), dim3(256), 0,
                       ctx->stream, (const float *)P, pstride, S, U, in.ldu, in.np, ncl);
}

// FP8 shapes per live bucket, timed like tile_choice (kind 3).
TileChoice tile_choice_fp8(l0l2_ctx *ctx, int64_t Kp) {
    Instance &in = ctx->inst;
    ensure_split(ctx, Kp, in.ldu, sizeof(float));
    if (ctx->force_xw >= 0) {
        // fixed shapes: 0-11 -> the unsliced register tile; the sliced ones to the
        // register tile in 4 slices (14, 16) or 8 (15), the 128 x 128 LDS-staged
        // tile in 4 slices (12, 13) or 8 (17)
        TileChoice f;
        const int x = ctx->force_xw;
        f.xw = x < kShapes ? 0 : x == 15 ? 2 : (x == 12 || x == 13) ? 3 : x == 17 ? 4 : 1;
        f.xtu = std::min(ctx->force_xtu, kShapesFp8 - 1);
        return f;
    }
    auto key = std::make_pair(3, Kp);
    auto it = in.tiles.find(key);
    if (it != in.tiles.end()) return it->second;
    TileChoice tc;
    tc.xw = tc.xtu = 0;
    if (ctx->tune) {
        hipStream_t s = ctx->stream;
        DevBuf inactive;
        inactive.ensure(sizeof(int) * Kp);
        HIPCHK(hipMemsetAsync(inactive.ptr, 0, sizeof(int) * Kp, s));
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        Sweep<float> s32 = sweep32(ctx);
        auto time_shape = [&](int v, int which, int reps) {
            HIPCHK(hipEventRecord(e0, s));
            for (int t = 0; t < reps; ++t) {
                if (which == 0) launch_xw_fp8(v, ctx, s32.W, s32.U, Kp, NodeCols{nullptr});
                else launch_xtu_fp8(v, ctx, Kp, inactive.as<int>(), 0, nullptr, NodeCols{nullptr});
            }
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            return ms / (float)reps;
        };
        // xw shape 0 always fits (node tile 32); a sliced one is a candidate
        // where its tile unsliced would leave compute units idle (fewer
        // workgroups than the 256 CUs); xtu shapes need their node tile
        auto valid = [&](int v, int which) {
            if (which == 1) return v < kShapesFp8 && Kp % kF8TN[v] == 0;
            if (v == 0) return true;
            return Kp % kF8XwT[v] == 0 && (in.np / kF8XwT[v]) * (Kp / kF8XwT[v]) < 256;
        };
        constexpr int NV = kShapesFp8Xw > kShapesFp8 ? kShapesFp8Xw : kShapesFp8;
        float t0 = 0.f;
        for (int v = 0; v < NV; ++v)
            for (int which = 0; which < 2; ++which)
                if (valid(v, which)) t0 = std::max(t0, time_shape(v, which, 1));
        const int reps = std::max(1, std::min(8, (int)(0.2f / std::max(t0, 1e-4f))));
        const int rounds = t0 > 1.0f ? 2 : 4;
        float best[NV][2];
        for (int v = 0; v < NV; ++v) best[v][0] = best[v][1] = 1e30f;
        for (int r = 0; r < rounds; ++r)
            for (int v = 0; v < NV; ++v)
                for (int which = 0; which < 2; ++which)
                    if (valid(v, which)) best[v][which] = std::min(best[v][which], time_shape(v, which, reps));
        for (int v = 1; v < NV; ++v) {
            if (valid(v, 0) && best[v][0] < best[tc.xw][0]) tc.xw = v;
            if (valid(v, 1) && best[v][1] < best[tc.xtu][1]) tc.xtu = v;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIPCHK(hipGetLastError());
    }
    if (!ctx->tune && big_batch_rule(in, Kp)) tc.xtu = 2;            // LDS-staged 128 x 128
    return in.tiles[key] = tc;
}

// One anchored sweep in FP8 storage: U = Xh d with the codes (register or
// LDS-staged tiles, as timed), then the FP64 update from z_a + Xh^T U.
void sweep_once_fp8(l0l2_ctx *ctx, int64_t Kp, bool store_b, int64_t active, bool gate) {
    Workspace &ws = ctx->ws;
    Sweep<float> s32 = sweep32(ctx);
    const NodeCols ncl = active_cols(ctx);
    const TileChoice tc = tile_choice_fp8(ctx, Kp);
    prof_begin(ctx, PROF_GEMM_XW_FP8);
    launch_xw_fp8(tc.xw, ctx, s32.W, s32.U, Kp, ncl);
    prof_end(ctx, PROF_GEMM_XW_FP8, active);
    prof_begin(ctx, PROF_ADMM_XTU_FP8);
    launch_xtu_fp8(tc.xtu, ctx, Kp, ws.active.as<int>(), store_b ? 1 : 0, gate ? ws.gpart.as<double>() : nullptr, ncl);
    prof_end(ctx, PROF_ADMM_XTU_FP8, active);
    HIPCHK(hipGetLastError());
}

DualArgs dual_args(const Instance &in) {
    DualArgs d;
    d.l0 = in.mp.l0; d.l2 = in.mp.l2; d.M = in.mp.M; d.s = in.mp.s;
    d.two_M_l2 = in.mp.two_M_l2; d.four_l2 = in.mp.four_l2; d.l2_M2 = in.mp.l2_M2; d.psi_lin = in.mp.psi_lin;
    const double u = 1.1102230246251565e-16;
    d.gamma_n = (double)in.n * u / (1.0 - (double)in.n * u);
    d.free_quad = in.mp.free_quad;
    d.p = in.p;
    return d;
}

// FP64 check at (B, beta) of type T: fills ws.lb / primal / status / active and
// the two counters (active nodes; active nodes above switch_tol), and in mode 0
// rebuilds the active list.  gated: only the nodes of the last gap estimate's
// check list are evaluated (the others stay active); otherwise every active
// node (mode 0) or every node of the padded batch (mode 1, bound only).
template <class T>
void check_once(l0l2_ctx *ctx, const T *B, const T *beta, int64_t Kp, double tol, double switch_tol, int mode,
                bool gated = false, int budget = 0) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    const int64_t np = in.np, pp = in.pp;
    const int64_t ntr = np / 32;
    NodeCols ncl{nullptr};
    if (mode == 0) ncl = gated ? NodeCols{ws.clist.as<int>()} : active_cols(ctx);
    // Tile of each FP64 product: 32 x 32 (8 waves) by default; once its grid
    // has at least 4 workgroups per CU at 64 nodes per workgroup, 64 x 64 (4
    // waves), which reads each panel of X a quarter as often per node.  The two
    // kernels choose separately (rows n of the first, p of the second): the
    // partial sums keep their 32-row and 32-coordinate layout either way.
    const bool wide_xr = Kp % 64 == 0 && np % 64 == 0 && ntr * (Kp / 64) >= 1024;
    const bool wide_xtr = Kp % 64 == 0 && pp % 64 == 0 && (pp / 32) * (Kp / 64) >= 1024;
    DualArgs da = dual_args(in);
    const T *bd = mode == 0 ? beta : B;
    auto launch_xr = [&](auto bm, auto bn, auto wv) {
        constexpr int BM = decltype(bm)::value, BN = decltype(bn)::value, WV = decltype(wv)::value;
        const dim3 g((unsigned)(np / (16 * BM)), (unsigned)(Kp / (16 * BN)), mode == 0 ? 2u : 1u);
        hipLaunchKernelGGL((k_check_xr<T, BM, BN, WV>), g, dim3(64 * WV), 0, s, in.X64R.as<double>(), in.ldxr, B,
                           beta, in.ldp, pp, in.y64.as<double>(), ws.R.as<double>(), in.ldu64,
                           ws.rpart.as<double>(), ncl);
    };
    auto launch_xtr = [&](auto bm, auto bn, auto wv) {
        constexpr int BM = decltype(bm)::value, BN = decltype(bn)::value, WV = decltype(wv)::value;
        const dim3 g((unsigned)(pp / (16 * BM)), (unsigned)(Kp / (16 * BN)));
        hipLaunchKernelGGL((k_dual_xtr<T, BM, BN, WV>), g, dim3(64 * WV), 0, s, in.X64.as<double>(), in.ldx,
                           ws.R.as<double>(), in.ldu64, np, ws.codes.as<uint8_t>(), bd, in.colnrm.as<double>(),
                           ws.rpart.as<double>(), ntr, ws.active.as<int>(), ws.part.as<double>(), in.ldp, da, ncl);
    };
    using I2 = std::integral_constant<int, 2>;
    using I4 = std::integral_constant<int, 4>;
    using I8 = std::integral_constant<int, 8>;
    prof_begin(ctx, PROF_CHECK);
    if (wide_xr) launch_xr(I4{}, I4{}, I4{});
    else launch_xr(I2{}, I2{}, I8{});
    if (wide_xtr) launch_xtr(I4{}, I4{}, I4{});
    else launch_xtr(I2{}, I2{}, I8{});
    FinArgs fa;
    const double u = 1.1102230246251565e-16;
    fa.gamma_n2 = ((double)in.n + 2.0) * u / (1.0 - ((double)in.n + 2.0) * u);
    fa.gamma_p = (double)in.p * u / (1.0 - (double)in.p * u);
    fa.tol = tol;
    fa.switch_tol = switch_tol;
    fa.K = Kp;
    fa.ntile = pp / 32;
    fa.ntr = ntr;
    fa.mode = mode;
    fa.budget = budget;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((Kp + 3) / 4)), dim3(256), 0, s, ws.rpart.as<double>(),
                       ws.part.as<double>(), ws.active.as<int>(), ws.status.as<int>(), ws.iters.as<int>(),
                       ws.lb.as<double>(), ws.primal.as<double>(), ws.counter.as<int>(), ws.nlist.as<int>(),
                       ws.ncount.as<int>(), ws.sweep_no.as<int>(), fa, gated ? ws.needs.as<int>() : nullptr,
                       ws.gest.as<double>(), ws.start.as<int>(), ws.dlist.as<int>());
    if (mode == 0)
        hipLaunchKernelGGL(k_list_commit, dim3(1), dim3(256), 0, s, ws.nlist.as<int>(), ws.ncount.as<int>(),
                           ws.list.as<int>(), ws.clist.as<int>(), Kp);
    prof_end(ctx, PROF_CHECK);
    HIPCHK(hipGetLastError());
}

template <class T>
void init_batch(l0l2_ctx *ctx, const Sweep<T> &sw, int64_t K, int64_t Kp) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(k_set_active, dim3((unsigned)((Kp + 255) / 256)), dim3(256), 0, s, ws.active.as<int>(),
                       ws.status.as<int>(), ws.iters.as<int>(), ws.list.as<int>(), ws.clist.as<int>(), K, Kp,
                       ws.sweep_no.as<int>(), ws.start.as<int>());
    hipLaunchKernelGGL((k_init<T>), dim3(grid1d(Kp * in.ldp)), dim3(256), 0, s, ws.codes.as<uint8_t>(), sw.beta,
                       sw.V, sw.W, sw.c, (T)in.mp.rho, in.ldp, Kp * in.ldp);
    HIPCHK(hipGetLastError());
}

// Continuous batching (node queue): slot pairs[2e] takes queue node pairs[2e+1]:
// its codes (FIX0 past p), its warm start (beta with F0 imposed, V) in the state
// type T, W = c + rho beta - V, and (promote) the FP64 state of the anchored
// sweeps; the slot becomes active with its sweep count starting now.
template <class T>
__global__ void k_queue_load(const uint8_t *__restrict__ qcodes, const T *__restrict__ qbeta,
                             const T *__restrict__ qv, int64_t p, const int *__restrict__ pairs, uint8_t *codes,
                             T *beta, T *V, T *W, const T *__restrict__ c, T rho, double *beta64, double *V64,
                             double *W64, const double *__restrict__ c64, double rho64, int promote, int64_t ldp,
                             int *active, int *status, int *iters, int *start, const int *__restrict__ sweep_no) {
    const int e = blockIdx.y;
    const int slot = pairs[2 * e], q = pairs[2 * e + 1];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < ldp) {
        const int64_t o = (int64_t)slot * ldp + j;
        const uint8_t code = j < p ? qcodes[(int64_t)q * p + j] : (uint8_t)CODE_FIX0;
        const T b = (j < p && code != CODE_FIX0) ? qbeta[(int64_t)q * p + j] : T(0);
        const T v = j < p ? qv[(int64_t)q * p + j] : T(0);
        codes[o] = code;
        beta[o] = b;
        V[o] = v;
        W[o] = c[j] + rho * b - v;
        if (promote) {
            beta64[o] = (double)b;
            V64[o] = (double)v;
            W64[o] = c64[j] + rho64 * (double)b - (double)v;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        active[slot] = 1;
        status[slot] = 1;
        iters[slot] = 0;
        start[slot] = *sweep_no;
    }
}

// The results of retired slots to their queue positions: lb, primal, sweeps,
// status, and the final (beta, V) in the output type TO from the state of the
// slot (the FP64 state of anchored sweeps, or the state itself).
template <class TS, class TO>
__global__ void k_queue_store(const int *__restrict__ pairs, const TS *__restrict__ beta, const TS *__restrict__ V,
                              int64_t ldp, int64_t p, const double *__restrict__ lb, const double *__restrict__ primal,
                              const int *__restrict__ iters, const int *__restrict__ status, TO *__restrict__ qbeta,
                              TO *__restrict__ qv, double *__restrict__ qlb, double *__restrict__ qprimal,
                              int *__restrict__ qiters, int *__restrict__ qstatus) {
    const int e = blockIdx.y;
    const int slot = pairs[2 * e], q = pairs[2 * e + 1];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < p) {
        qbeta[(int64_t)q * p + j] = (TO)beta[(int64_t)slot * ldp + j];
        qv[(int64_t)q * p + j] = (TO)V[(int64_t)slot * ldp + j];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        qlb[q] = lb[slot];
        qprimal[q] = primal[slot];
        qiters[q] = iters[slot];
        qstatus[q] = status[slot];
    }
}

// Appends m slots to the active list after its first `base` entries.
__global__ void k_list_append(int *list, int64_t base, const int *__restrict__ pairs, int m) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) list[base + e] = pairs[2 * e];
}

enum SweepKind { SK_F32 = 0, SK_F64 = 1, SK_BF16 = 2, SK_ANCH = 3 };

// One block: `n` sweeps of the given kind, then the FP64 gap check and the
// read-back of the two counters into pinned host memory.  Issued eagerly.
// Unless force is set, the last sweep also forms the gap estimate and the exact
// check evaluates only the nodes that may pass the tolerance; the others stay
// active and are counted above switch_tol by their estimate.
// Node columns a block's sweep launches cover: the active count rounded up to a
// power of two (at least 32, at most the padded batch).  Tile shapes are tuned
// per such bucket, since the best shape for a few live nodes is not the best
// for a full batch.  Fixed shapes (l0l2_set_tiles) always cover the whole batch.
int64_t live_bucket(const l0l2_ctx *ctx, int64_t active, int64_t Kp) {
    if (ctx->force_xw >= 0) return Kp;
    int64_t b = kPadNodes;
    while (b < active) b *= 2;
    return std::min(b, Kp);
}

// A block of sweeps in three parts (its start, sweep t, its end), so that the
// cross-instance executor can interleave the blocks of several instances.
struct BlockPlan {
    int64_t cols = 0;   // node columns of the launches: the live count rounded up (live_bucket)
    bool gram = false;  // Gram form of the b-update
};

BlockPlan block_begin(l0l2_ctx *ctx, int kind, int64_t Kp, int n, int64_t active) {
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    BlockPlan bp;
    bp.cols = live_bucket(ctx, active, Kp);
    hipLaunchKernelGGL(k_sweep_add, dim3(1), dim3(1), 0, s, ws.sweep_no.as<int>(), n, ws.gate.as<int>(),
                       ws.ncount.as<int>(), ws.counter.as<int>());
    bp.gram = (kind == SK_F32 || kind == SK_BF16 || kind == SK_ANCH) && gram_form(ctx);
    if (bp.gram) ensure_gram(ctx);
    if (kind == SK_ANCH) {
        if (bp.gram) anchor_start_gram(ctx, Kp, bp.cols);
        else anchor_start(ctx, Kp, bp.cols);
    }
    return bp;
}

void block_sweep(l0l2_ctx *ctx, int kind, const BlockPlan &bp, int t, int n, bool force, int64_t active) {
    Instance &in = ctx->inst;
    const int64_t cols = bp.cols;
    const bool last = t == n, gate = last && !force, gram = bp.gram;
    if (gram && kind == SK_F32) sweep_once_gram(ctx, cols, last, active, gate, t);
    else if (gram && in.prec == L0L2_BF16) sweep_once_bf16_gram(ctx, cols, last, active, gate, kind == SK_ANCH, t);
    else if (gram) sweep_once_anch_gram(ctx, cols, last, active, gate, t);
    else if (kind == SK_F64) sweep_once<double>(ctx, sweep64(ctx), cols, last, active, gate);
    else if (kind == SK_BF16) sweep_once_bf16(ctx, cols, last, active, gate, false);
    else if (kind == SK_ANCH && in.prec == L0L2_BF16) sweep_once_bf16(ctx, cols, last, active, gate, true);
    else if (kind == SK_ANCH && in.prec == L0L2_FP8) sweep_once_fp8(ctx, cols, last, active, gate);
    else if (kind == SK_ANCH) sweep_once_anch(ctx, cols, last, active, gate);
    else sweep_once<float>(ctx, sweep32(ctx), cols, last, active, gate);
}

void block_end(l0l2_ctx *ctx, int kind, const BlockPlan &bp, int64_t Kp, int n, double tol, double switch_tol,
               bool force, int budget) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    const int64_t cols = bp.cols;
    // an odd Gram-form block leaves the latest W in the second buffer (a node that
    // retires keeps a stale W in it, which nothing reads again)
    if (bp.gram && (kind == SK_F32 || kind == SK_BF16) && (n & 1))
        HIPCHK(hipMemcpyAsync(ws.W.ptr, ws.W2.ptr, sizeof(float) * Kp * in.ldp, hipMemcpyDeviceToDevice, s));
    if (!force) {
        int rows = 32;
        if (kind == SK_F64) rows = kTileTM[tile_choice<double>(ctx, sweep64(ctx), cols).xtu];
        else if (kind == SK_BF16 || (kind == SK_ANCH && in.prec == L0L2_BF16))
            rows = kBfTM[tile_choice_bf16(ctx, cols).xtu];
        else if (kind == SK_ANCH && in.prec == L0L2_FP8) rows = kF8TM[tile_choice_fp8(ctx, cols).xtu];
        else rows = kTileTM[tile_choice<float>(ctx, sweep32(ctx), cols).xtu];
        // single-term blocks before the switch: their gaps sit above the FP32
        // floor, so an exact check there would almost never retire a node
        const int skip = kind == SK_BF16 && bf16_single(ctx, cols) ? 1 : 0;
        GateFin gf{in.yy, tol, Kp, in.pp / rows, budget, skip};
        prof_begin(ctx, PROF_CHECK);
        hipLaunchKernelGGL(k_gate, dim3((unsigned)((Kp + 3) / 4)), dim3(256), 0, s, ws.gpart.as<double>(),
                           ws.active.as<int>(), ws.needs.as<int>(), ws.gest.as<double>(), ws.clist.as<int>(),
                           ws.gate.as<int>(), gf, (const int *)ws.sweep_no.ptr, (const int *)ws.start.ptr);
        prof_end(ctx, PROF_CHECK);
        HIPCHK(hipGetLastError());
    }
    if (kind == SK_F64 || kind == SK_ANCH) {
        Sweep<double> sw = sweep64(ctx);
        check_once<double>(ctx, sw.B, sw.beta, Kp, tol, switch_tol, 0, !force, budget);
    } else {
        Sweep<float> sw = sweep32(ctx);
        check_once<float>(ctx, sw.B, sw.beta, Kp, tol, switch_tol, 0, !force, budget);
    }
    HIPCHK(hipMemcpyAsync(ws.host_counter, ws.counter.ptr, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
}

void issue_block(l0l2_ctx *ctx, int kind, int64_t Kp, int n, double tol, double switch_tol, int64_t active,
                 bool force, int budget) {
    const BlockPlan bp = block_begin(ctx, kind, Kp, n, active);
    for (int t = 1; t <= n; ++t) block_sweep(ctx, kind, bp, t, n, force, active);
    block_end(ctx, kind, bp, Kp, n, tol, switch_tol, force, budget);
}

// ---------------------------------------------------------------------------
// Batching across instances.  Contexts attached to an executor (the server's)
// hand each block of sweeps to it instead of replaying their own graph.  The
// executor takes every block waiting when it becomes free, issues their starts,
// then sweep t of all of them together, then their ends, on its own stream, and
// hands each context its counters.  The sweeps whose contractions use the
// 32 x 32 register tile (FP32 mode and the BF16 split form in both b-update
// forms and both phases, FP64 mode) go out as grouped launches, one per
// contraction kind, whose
// workgroups are the tiles of every member; the other sweeps are issued for
// their context alone, between them.  Instances join and leave between blocks
// (continuous batching).  A member's tiles compute what its own launch would,
// so results do not depend on what else runs.
// ---------------------------------------------------------------------------
enum GroupClass { GC_NONE, GC_F32, GC_F32_GRAM, GC_F64, GC_ANCH, GC_ANCH_GRAM, GC_BF, GC_BF_GRAM, GC_BFA, GC_BFA_GRAM };

GroupClass group_class(l0l2_ctx *ctx, int kind, const BlockPlan &bp) {
    const Instance &in = ctx->inst;
    if (kind == SK_F64) {
        const TileChoice &tc = tile_choice<double>(ctx, sweep64(ctx), bp.cols);
        return tc.xw == 0 && tc.xtu == 0 ? GC_F64 : GC_NONE;
    }
    if (in.prec == L0L2_BF16 && (kind == SK_BF16 || kind == SK_ANCH)) {
        // the BF16 split form on the register tile (the single-term blocks need
        // the LDS-staged tiles, so they are not taken here)
        const TileChoice &tc = tile_choice_bf16(ctx, bp.cols);
        if (tc.xtu != 0 || (!bp.gram && tc.xw != 0)) return GC_NONE;
        if (kind == SK_BF16) return bp.gram ? GC_BF_GRAM : GC_BF;
        return bp.gram ? GC_BFA_GRAM : GC_BFA;
    }
    if (in.prec != L0L2_FP32 || (kind != SK_F32 && kind != SK_ANCH)) return GC_NONE;
    const TileChoice &tc = tile_choice<float>(ctx, sweep32(ctx), bp.cols);
    if (tc.xtu != 0 || (!bp.gram && tc.xw != 0)) return GC_NONE;
    if (kind == SK_F32) return bp.gram ? GC_F32_GRAM : GC_F32;
    return bp.gram ? GC_ANCH_GRAM : GC_ANCH;
}

// The members of one grouped launch kind, flushed when full.
template <class M>
struct GroupBatch {
    Group<M> g{};
    int tiles = 0;
    int64_t *launches, *members;
    void (*go)(const Group<M> &, int, hipStream_t);
    void add(const M &m, int ntiles, hipStream_t s) {
        if (g.count == kGroupMax) flush(s);
        g.m[g.count] = m;
        g.m[g.count].tile0 = tiles;
        ++g.count;
        tiles += ntiles;
    }
    void flush(hipStream_t s) {
        if (!g.count) return;
        go(g, tiles, s);
        ++*launches;
        *members += g.count;
        g.count = 0;
        tiles = 0;
    }
};

template <class T>
void go_xw(const Group<XwMember<T>> &g, int tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_gemm_xw_grp<T>, dim3((unsigned)tiles), dim3(256), 0, s, g);
}
template <class T>
void go_xtu(const Group<XtuMember<T>> &g, int tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_admm_xtu_grp<T>, dim3((unsigned)tiles), dim3(256), 0, s, g);
}
void go_anch(const Group<AnchMember> &g, int tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_admm_xtu_anch_grp, dim3((unsigned)tiles), dim3(256), 0, s, g);
}
void go_xw_bf(const Group<XwBfMember> &g, int tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_gemm_xw_bf16_grp, dim3((unsigned)tiles), dim3(64 * kWavesBf16), 0, s, g);
}
void go_xtu_bf(const Group<XtuBfMember> &g, int tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_admm_xtu_bf16_grp, dim3((unsigned)tiles), dim3(64 * kWavesBf16), 0, s, g);
}
void go_anch_bf(const Group<AnchBfMember> &g, int tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_admm_xtu_anch_bf16_grp, dim3((unsigned)tiles), dim3(64 * kWavesBf16), 0, s, g);
}

template <class T>
XwMember<T> xw_member(const Sweep<T> &sw, const Instance &in, const int *cols, int64_t ncols, int &ntiles) {
    XwMember<T> m{};
    m.A = sw.XhR; m.lda = sw.ldr; m.B = sw.W; m.ldb = sw.ldp; m.U = sw.U; m.ldu = sw.ldu; m.kdim = in.pp;
    m.cols = cols;
    m.gx = (int)(in.np / 32);
    ntiles = m.gx * (int)(ncols / 32);
    return m;
}

struct GroupReq {
    l0l2_ctx *ctx;
    int kind;
    int64_t Kp;
    int n;
    double tol, switch_tol;
    int64_t active;
    bool force;
    int budget;
    int out[3] = {0, 0, 0};
    bool done = false;
    int rc = L0L2_OK;
    std::string err;
};

}  // namespace

struct GroupExec {
    int device = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<GroupReq *> pending;
    int attached = 0;   // contexts attached (each has at most one block pending)
    bool stop = false;
    std::thread th;
    GroupStats st;
};

namespace {

// The ctx's work goes to the executor's stream (and its allocations are
// charged to the ctx) while the executor issues for it.
struct OnExec {
    l0l2_ctx *ctx;
    hipStream_t saved;
    MemCount *mem_saved;
    OnExec(l0l2_ctx *c, hipStream_t s) : ctx(c), saved(c->stream), mem_saved(thread_mem()) {
        c->stream = s;
        thread_mem() = &c->mem;
    }
    ~OnExec() {
        ctx->stream = saved;
        thread_mem() = mem_saved;
    }
};

GroupStats run_group(GroupExec &ex, std::vector<GroupReq *> &batch) {
    hipStream_t S = ex.stream;
    GroupStats st;
    const size_t m = batch.size();
    std::vector<BlockPlan> plan(m);
    std::vector<GroupClass> cls(m, GC_NONE);
    std::vector<char> ok(m, 1);
    auto guard = [&](size_t i, auto &&f) {
        if (!ok[i]) return;
        OnExec on(batch[i]->ctx, S);
        try {
            f();
        } catch (const Error &e) {
            ok[i] = 0;
            batch[i]->rc = e.code;
            batch[i]->err = e.msg;
        } catch (const std::exception &e) {
            ok[i] = 0;
            batch[i]->rc = L0L2_E_DEVICE;
            batch[i]->err = e.what();
        }
    };
    int nmax = 0;
    for (size_t i = 0; i < m; ++i) {
        GroupReq &r = *batch[i];
        guard(i, [&] {
            HIPCHK(hipStreamWaitEvent(S, r.ctx->ev_group, 0));
            plan[i] = block_begin(r.ctx, r.kind, r.Kp, r.n, r.active);
            cls[i] = group_class(r.ctx, r.kind, plan[i]);
        });
        if (ok[i]) nmax = std::max(nmax, r.n);
    }
    GroupBatch<XwMember<float>> xw32{{}, 0, &st.launches, &st.members, go_xw<float>};
    GroupBatch<XwMember<double>> xw64{{}, 0, &st.launches, &st.members, go_xw<double>};
    GroupBatch<XtuMember<float>> xtu32{{}, 0, &st.launches, &st.members, go_xtu<float>};
    GroupBatch<XtuMember<double>> xtu64{{}, 0, &st.launches, &st.members, go_xtu<double>};
    GroupBatch<AnchMember> anch{{}, 0, &st.launches, &st.members, go_anch};
    GroupBatch<XwBfMember> xwbf{{}, 0, &st.launches, &st.members, go_xw_bf};
    GroupBatch<XtuBfMember> xtubf{{}, 0, &st.launches, &st.members, go_xtu_bf};
    GroupBatch<AnchBfMember> anchbf{{}, 0, &st.launches, &st.members, go_anch_bf};
    for (int t = 1; t <= nmax; ++t) {
        bool xtu_pending = false;
        for (size_t i = 0; i < m; ++i) {
            GroupReq &r = *batch[i];
            if (!ok[i] || t > r.n) continue;
            l0l2_ctx *ctx = r.ctx;
            if (cls[i] == GC_NONE) {
                guard(i, [&] { block_sweep(ctx, r.kind, plan[i], t, r.n, r.force, r.active); });
                continue;
            }
            guard(i, [&] {
                Instance &in = ctx->inst;
                Workspace &ws = ctx->ws;
                const bool last = t == r.n, gate = last && !r.force;
                const int64_t ncols = plan[i].cols;
                const int *cols = ws.list.as<int>();
                const int gy = (int)(ncols / 32), gxp = (int)(in.pp / 32);
                int nt = 0;
                // a member's contraction over n waits for its contraction over p:
                // flush the pending contractions over p before an XTU group fills
                auto before_xtu = [&] {
                    if (xtu32.g.count == kGroupMax || xtu64.g.count == kGroupMax || anch.g.count == kGroupMax ||
                        xtubf.g.count == kGroupMax || anchbf.g.count == kGroupMax) {
                        xw32.flush(S);
                        xw64.flush(S);
                        xwbf.flush(S);
                    }
                };
                if (cls[i] == GC_BF || cls[i] == GC_BF_GRAM || cls[i] == GC_BFA || cls[i] == GC_BFA_GRAM) {
                    const Sweep<float> s32 = sweep32(ctx);
                    const bool gram = cls[i] == GC_BF_GRAM || cls[i] == GC_BFA_GRAM;
                    const bool anchd = cls[i] == GC_BFA || cls[i] == GC_BFA_GRAM;
                    // the contraction over n (over p with G): A, its range, the node
                    // operand read and the one written
                    const __bf16 *hi = gram ? in.Ghi.as<__bf16>() : in.Xh.as<__bf16>();
                    const __bf16 *lo = gram ? in.Glo.as<__bf16>() : in.XhLo.as<__bf16>();
                    const int64_t lda = gram ? in.ldgb : in.ldw, ldu = gram ? in.ldp : in.ldu;
                    const int64_t kdim = gram ? in.pp : in.np;
                    const float *U = gram ? gram_in(ctx, t) : s32.U;
                    float *wout = gram ? gram_out(ctx, t) : s32.W;
                    if (!gram) {
                        XwBfMember x{};
                        x.hi = in.XhR.as<__bf16>(); x.lo = in.XhRLo.as<__bf16>(); x.lda = in.ldwr;
                        x.B = s32.W; x.ldb = in.ldp; x.U = s32.U; x.ldu = in.ldu; x.kdim = in.pp; x.cols = cols;
                        x.gx = (int)(in.np / 32);
                        xwbf.add(x, x.gx * gy, S);
                    }
                    before_xtu();
                    if (anchd) {
                        const Sweep<double> s64 = sweep64(ctx);
                        AnchBfMember a{};
                        a.hi = hi; a.lo = lo; a.lda = lda; a.U = U; a.ldu = ldu; a.kdim = kdim;
                        a.Za = ws.Za.as<double>(); a.Wa = ws.Wa.as<double>();
                        a.W = s64.W; a.beta = s64.beta; a.V = s64.V; a.Bst = s64.B; a.d = wout; a.c = s64.c;
                        a.codes = ws.codes.as<uint8_t>(); a.active = ws.active.as<int>(); a.cols = cols;
                        a.gpart = gate ? ws.gpart.as<double>() : nullptr; a.ldp = in.ldp; a.store_b = last ? 1 : 0;
                        a.gx = gxp; a.q = dev_params<double>(in.mp); a.ga = gate_args(in);
                        anchbf.add(a, gxp * gy, S);
                    } else {
                        XtuBfMember x{};
                        x.hi = hi; x.lo = lo; x.lda = lda; x.U = U; x.ldu = ldu; x.kdim = kdim;
                        x.W = gram ? gram_in(ctx, t) : s32.W; x.Wout = wout;
                        x.beta = s32.beta; x.V = s32.V; x.Bst = s32.B; x.c = s32.c;
                        x.codes = ws.codes.as<uint8_t>(); x.active = ws.active.as<int>(); x.cols = cols;
                        x.gpart = gate ? ws.gpart.as<double>() : nullptr; x.ldp = in.ldp; x.store_b = last ? 1 : 0;
                        x.gx = gxp; x.q = dev_params<float>(in.mp); x.ga = gate_args(in);
                        xtubf.add(x, gxp * gy, S);
                    }
                } else if (cls[i] == GC_F64) {
                    const Sweep<double> sw = sweep64(ctx);
                    xw64.add(xw_member<double>(sw, in, cols, ncols, nt), nt, S);
                    XtuMember<double> x{};
                    x.A = sw.Xh; x.lda = sw.ldc; x.U = sw.U; x.ldu = sw.ldu; x.kdim = in.np;
                    x.W = sw.W; x.Wout = sw.W; x.beta = sw.beta; x.V = sw.V; x.Bst = sw.B; x.c = sw.c;
                    x.codes = ws.codes.as<uint8_t>(); x.active = ws.active.as<int>(); x.cols = cols;
                    x.gpart = gate ? ws.gpart.as<double>() : nullptr; x.ldp = sw.ldp; x.store_b = last ? 1 : 0;
                    x.gx = gxp; x.q = dev_params<double>(in.mp); x.ga = gate_args(in);
                    before_xtu();
                    xtu64.add(x, gxp * gy, S);
                } else if (cls[i] == GC_F32 || cls[i] == GC_F32_GRAM) {
                    Sweep<float> sw = sweep32(ctx);
                    float *wout = sw.W;
                    if (cls[i] == GC_F32_GRAM) {
                        sw.Xh = in.G32.as<float>();
                        sw.ldc = in.ldg32;
                        sw.W = gram_in(ctx, t);
                        sw.U = sw.W;
                        sw.ldu = in.ldp;
                        wout = gram_out(ctx, t);
                    } else {
                        xw32.add(xw_member<float>(sw, in, cols, ncols, nt), nt, S);
                    }
                    XtuMember<float> x{};
                    x.A = sw.Xh; x.lda = sw.ldc; x.U = sw.U; x.ldu = sw.ldu;
                    x.kdim = cls[i] == GC_F32_GRAM ? in.pp : in.np;
                    x.W = sw.W; x.Wout = wout; x.beta = sw.beta; x.V = sw.V; x.Bst = sw.B; x.c = sw.c;
                    x.codes = ws.codes.as<uint8_t>(); x.active = ws.active.as<int>(); x.cols = cols;
                    x.gpart = gate ? ws.gpart.as<double>() : nullptr; x.ldp = sw.ldp; x.store_b = last ? 1 : 0;
                    x.gx = gxp; x.q = dev_params<float>(in.mp); x.ga = gate_args(in);
                    before_xtu();
                    xtu32.add(x, gxp * gy, S);
                } else {
                    Sweep<float> s32 = sweep32(ctx);
                    const Sweep<double> s64 = sweep64(ctx);
                    AnchMember a{};
                    if (cls[i] == GC_ANCH_GRAM) {
                        a.A = in.G32.as<float>(); a.lda = in.ldg32; a.U = gram_in(ctx, t); a.ldu = in.ldp;
                        a.kdim = in.pp; a.d = gram_out(ctx, t);
                    } else {
                        xw32.add(xw_member<float>(s32, in, cols, ncols, nt), nt, S);
                        a.A = s32.Xh; a.lda = s32.ldc; a.U = s32.U; a.ldu = s32.ldu; a.kdim = in.np; a.d = s32.W;
                    }
                    a.Za = ws.Za.as<double>(); a.Wa = ws.Wa.as<double>();
                    a.W = s64.W; a.beta = s64.beta; a.V = s64.V; a.Bst = s64.B; a.c = s64.c;
                    a.codes = ws.codes.as<uint8_t>(); a.active = ws.active.as<int>(); a.cols = cols;
                    a.gpart = gate ? ws.gpart.as<double>() : nullptr; a.ldp = s32.ldp; a.store_b = last ? 1 : 0;
                    a.gx = gxp; a.q = dev_params<double>(in.mp); a.ga = gate_args(in);
                    before_xtu();
                    anch.add(a, gxp * gy, S);
                }
                xtu_pending = true;
            });
        }
        xw32.flush(S);
        xw64.flush(S);
        xwbf.flush(S);
        if (xtu_pending) {
            xtu32.flush(S);
            xtu64.flush(S);
            anch.flush(S);
            xtubf.flush(S);
            anchbf.flush(S);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            for (size_t i = 0; i < m; ++i)
                if (ok[i]) {
                    ok[i] = 0;
                    batch[i]->rc = L0L2_E_DEVICE;
                    batch[i]->err = std::string("grouped sweep launch: ") + hipGetErrorString(e);
                }
    }
    for (size_t i = 0; i < m; ++i) {
        GroupReq &r = *batch[i];
        guard(i, [&] { block_end(r.ctx, r.kind, plan[i], r.Kp, r.n, r.tol, r.switch_tol, r.force, r.budget); });
    }
    const hipError_t e = hipStreamSynchronize(S);
    st.rounds = 1;
    st.blocks = (int64_t)m;
    for (size_t i = 0; i < m; ++i) {
        GroupReq &r = *batch[i];
        if (e != hipSuccess && ok[i]) {
            ok[i] = 0;
            r.rc = L0L2_E_DEVICE;
            r.err = std::string("executor stream: ") + hipGetErrorString(e);
        }
        if (ok[i])
            for (int k = 0; k < 3; ++k) r.out[k] = r.ctx->ws.host_counter[k];
    }
    return st;
}

// A round starts once every attached context has a block waiting, or
// kGroupWindowUs after the first one arrived: contexts released by the same
// round come back within microseconds (they only read their counters), while
// one busy with the end of its node batch (rounding, refinement, the next
// batch's assembly) is not waited for.
constexpr int kGroupWindowUs = 200;

void group_loop(GroupExec *ex) {
    (void)hipSetDevice(ex->device);
    for (;;) {
        std::vector<GroupReq *> batch;
        {
            std::unique_lock<std::mutex> lk(ex->mu);
            ex->cv.wait(lk, [&] { return ex->stop || !ex->pending.empty(); });
            if (ex->pending.empty()) break;
            const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(kGroupWindowUs);
            ex->cv.wait_until(lk, until, [&] { return ex->stop || (int)ex->pending.size() >= ex->attached; });
            batch.assign(ex->pending.begin(), ex->pending.end());
            ex->pending.clear();
        }
        const GroupStats d = run_group(*ex, batch);
        {
            std::lock_guard<std::mutex> lk(ex->mu);
            for (GroupReq *r : batch) r->done = true;
            ex->st.rounds += d.rounds;
            ex->st.blocks += d.blocks;
            ex->st.launches += d.launches;
            ex->st.members += d.members;
        }
        ex->cv_done.notify_all();
    }
}

// The block through the context's executor: waits for the round that runs it.
void group_run_block(l0l2_ctx *ctx, int kind, int64_t Kp, int n, double tol, double switch_tol, int64_t active,
                     bool force, int out[3], int budget) {
    GroupExec *ex = ctx->group;
    if (!ctx->ev_group) HIPCHK(hipEventCreateWithFlags(&ctx->ev_group, hipEventDisableTiming));
    // the executor's stream waits for what the context queued before the block
    HIPCHK(hipEventRecord(ctx->ev_group, ctx->stream));
    GroupReq r{ctx, kind, Kp, n, tol, switch_tol, active, force, budget};
    {
        std::lock_guard<std::mutex> lk(ex->mu);
        ex->pending.push_back(&r);
    }
    ex->cv.notify_one();
    {
        std::unique_lock<std::mutex> lk(ex->mu);
        ex->cv_done.wait(lk, [&] { return r.done; });
    }
    if (r.rc != L0L2_OK) fail(r.rc, r.err);
    out[0] = r.out[0];
    out[1] = r.out[1];
    out[2] = r.out[2];
}

}  // namespace

GroupExec *group_exec_create(int device) {
    auto ex = std::make_unique<GroupExec>();
    ex->device = device;
    HIPCHK(hipSetDevice(device));
    HIPCHK(hipStreamCreateWithFlags(&ex->stream, hipStreamNonBlocking));
    ex->th = std::thread(group_loop, ex.get());
    return ex.release();
}

void group_exec_destroy(GroupExec *ex) {
    if (!ex) return;
    {
        std::lock_guard<std::mutex> lk(ex->mu);
        ex->stop = true;
    }
    ex->cv.notify_all();
    if (ex->th.joinable()) ex->th.join();
    if (ex->stream) (void)hipStreamDestroy(ex->stream);
    delete ex;
}

void group_exec_attach(GroupExec *ex, int delta) {
    {
        std::lock_guard<std::mutex> lk(ex->mu);
        ex->attached += delta;
    }
    ex->cv.notify_all();
}

GroupStats group_exec_stats(GroupExec *ex) {
    std::lock_guard<std::mutex> lk(ex->mu);
    return ex->st;
}

namespace {

// Run one block and return the counters.  Blocks are captured once into a HIP
// graph per (kind, padded batch, block length, tolerances) and replayed; with
// the profiler on they are issued eagerly so each launch can be timed.
void run_block(l0l2_ctx *ctx, int kind, int64_t Kp, int n, double tol, double switch_tol, int64_t active,
               bool force, int out[3], int budget = 0) {
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    ++ws.stat_blocks;
    ws.stat_node_blocks += active;
    if (8 * active < Kp) ++ws.stat_sparse;
    if (ctx->group && !ctx->prof.on) {
        group_run_block(ctx, kind, Kp, n, tol, switch_tol, active, force, out, budget);
        return;
    }
    if (!ctx->use_graphs || ctx->prof.on) {
        issue_block(ctx, kind, Kp, n, tol, switch_tol, active, force, budget);
    } else {
        const int64_t cols = live_bucket(ctx, active, Kp);
        // settle the tile shapes first (the autotuner synchronises, and may grow
        // the split buffer, which drops the captured graphs)
        const bool bf = ctx->inst.prec == L0L2_BF16, f8 = ctx->inst.prec == L0L2_FP8;
        if ((kind == SK_F32 || kind == SK_BF16 || kind == SK_ANCH) && gram_form(ctx)) ensure_gram(ctx);   // not under capture
        if (kind == SK_F64 || kind == SK_ANCH) (void)tile_choice<double>(ctx, sweep64(ctx), cols);
        if (kind == SK_F32 || (kind == SK_ANCH && !bf && !f8)) (void)tile_choice<float>(ctx, sweep32(ctx), cols);
        if (kind == SK_BF16 || (kind == SK_ANCH && bf)) (void)tile_choice_bf16(ctx, cols);
        if (kind == SK_ANCH && f8) (void)tile_choice_fp8(ctx, cols);
        GraphKey key{kind, Kp, cols, n, force ? 1 : 0, tol, switch_tol, ws.gen, budget};
        auto it = ctx->graphs.find(key);
        if (it == ctx->graphs.end()) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ex = nullptr;
            if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                bool ok = true;
                try {
                    issue_block(ctx, kind, Kp, n, tol, switch_tol, active, force, budget);
                } catch (...) {
                    ok = false;
                }
                hipError_t e = hipStreamEndCapture(s, &g);
                if (ok && e == hipSuccess && g && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess)
                    ex = nullptr;
                if (g) (void)hipGraphDestroy(g);
            }
            (void)hipGetLastError();
            if (!ex) {
                // capture is not available here: issue blocks launch by launch from now on
                ctx->use_graphs = false;
                issue_block(ctx, kind, Kp, n, tol, switch_tol, active, force, budget);
                HIPCHK(hipStreamSynchronize(s));
                out[0] = ws.host_counter[0];
                out[1] = ws.host_counter[1];
                out[2] = ws.host_counter[2];
                return;
            }
            it = ctx->graphs.emplace(key, ex).first;
        }
        HIPCHK(hipGraphLaunch(it->second, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    out[0] = ws.host_counter[0];
    out[1] = ws.host_counter[1];
    out[2] = ws.host_counter[2];
}

// Single-precision-type solve (FP64 mode).
template <class T>
void solve_plain(l0l2_ctx *ctx, const Sweep<T> &sw, int K, const l0l2_admm_opts &o) {
    const int64_t Kp = round_up(K, kPadNodes);
    init_batch<T>(ctx, sw, K, Kp);
    const int m = std::max(1, o.check_every);
    int cnt[3];
    int64_t active = K;
    for (int t = 0; t < o.max_iter;) {
        check_cancel(ctx);
        const int n = std::min(m, o.max_iter - t);
        run_block(ctx, sizeof(T) == 8 ? SK_F64 : SK_F32, Kp, n, o.tol_node, o.tol_node, active,
                  t + n >= o.max_iter, cnt);
        t += n;
        active = cnt[0];
        if (cnt[0] == 0) break;
    }
}

// The b-update form by measurement (Sec. 3.1.1 offers both the p x p matrix
// D and the Woodbury form): on the instance's first solve with the Gram form a
// candidate, one sweep of each form is timed on the padded batch with every
// node masked (the products run, the epilogues write nothing), best of three
// rounds after a warm-up; the faster form is kept for the instance, and G is
// freed when the folded form wins.  BF16 mode times its Gram sweeps as they
// run: a block of ten is one split-form sweep and nine single-term sweeps
// where the LDS-staged tiles are chosen.
void decide_form(l0l2_ctx *ctx, int64_t Kp) {
    Instance &in = ctx->inst;
    if (in.form_pick || ctx->bform != 0 || !gram_candidate(in) || !ctx->tune) return;
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    ensure_gram(ctx);
    const bool bf = in.prec == L0L2_BF16;
    Sweep<float> s32 = sweep32(ctx);
    const DevParams<float> q32 = dev_params<float>(in.mp);
    // settle the tile shapes (their autotuner synchronises) before timing
    const TileChoice tcf = bf ? tile_choice_bf16(ctx, Kp) : tile_choice<float>(ctx, s32, Kp);
    HIPCHK(hipMemsetAsync(ws.active.ptr, 0, sizeof(int) * Kp, s));
    const int *inactive = ws.active.as<int>();
    const NodeCols all{nullptr};
    auto folded = [&] {
        if (bf) {
            launch_xw_bf16(tcf.xw, ctx, s32.W, s32.U, Kp, all);
            launch_xtu_bf16(tcf.xtu, ctx, false, Kp, inactive, 0, nullptr, all);
        } else {
            launch_xw<float, float, float>(tcf.xw, s, s32.XhR, s32.ldr, s32.W, s32.ldp, s32.U, s32.ldu, in.np, Kp,
                                           in.pp, all, split_buf(ctx));
            launch_xtu<float>(tcf.xtu, s, s32, in.np, in.pp, Kp, ws.codes.as<uint8_t>(), inactive, q32, 0);
        }
    };
    const bool single = bf && ctx->bf16_terms == 1 && tcf.xtu >= 1;
    auto gram_split = [&] {
        if (bf) {
            const GramBf gr{in.Ghi.as<__bf16>(), in.Glo.as<__bf16>(), in.ldgb, ws.W.as<float>(), ws.W2.as<float>()};
            launch_xtu_bf16(tcf.xtu, ctx, false, Kp, inactive, 0, nullptr, all, &gr);
        } else {
            Sweep<float> g = s32;
            g.Xh = in.G32.as<float>();
            g.ldc = in.ldg32;
            g.U = g.W;
            g.ldu = in.ldp;
            launch_xtu<float>(tcf.xtu, s, g, in.pp, in.pp, Kp, ws.codes.as<uint8_t>(), inactive, q32, 0, nullptr,
                              GateArgs{}, all, ws.W2.as<float>());
        }
    };
    auto gram_single = [&] { launch_xtu_bf16s(tcf.xtu, ctx, 1, Kp, 0, nullptr, all, 2); };
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto time_ms = [&](auto &&f) {
        f();   // warm-up
        float best = 1e30f;
        for (int r = 0; r < 3; ++r) {
            HIPCHK(hipEventRecord(e0, s));
            f();
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        return (double)best;
    };
    in.form_ms[0] = time_ms(folded);
    in.form_ms[1] = single ? 0.1 * time_ms(gram_split) + 0.9 * time_ms(gram_single) : time_ms(gram_split);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipGetLastError());
    in.form_pick = in.form_ms[1] < in.form_ms[0] ? 2 : 1;
    if (in.form_pick == 1) {
        in.G64.release();
        in.G32.release();
        in.Ghi.release();
        in.Glo.release();
        in.gram_built = false;
    }
    drop_graphs(ctx);   // any block captured before the decision took the assumed form
}

// Mixed precision (FP32 state): reduced-precision sweeps (FP32, or the BF16
// form) while the batch converges, then anchored sweeps (FP64 state, the
// reduced products act on the movement since each block's FP64 anchor) from the
// FP32 iterates.  The plain reduced sweeps stop for the batch once every active
// node's gap is below switch_tol (50 tol_node for FP32 and the BF16 single-term
// blocks, 200 tol_node for the BF16 split form: the measured floors are about
// 1e-6..5e-6 and 1e-4), or the number of nodes
// above it has not dropped for 5 checks, or half the sweep budget is spent.
// FP8 storage has no plain phase (its floor is far above any useful gap): its
// sweeps are anchored from the start.  Bounds are FP64 throughout; the final
// iterates are returned in FP32.
void solve_mixed(l0l2_ctx *ctx, int K, const l0l2_admm_opts &o) {
    Instance &in = ctx->inst;
    const int64_t Kp = round_up(K, kPadNodes);
    decide_form(ctx, Kp);
    Sweep<float> s32 = sweep32(ctx);
    Sweep<double> s64 = sweep64(ctx);
    init_batch<float>(ctx, s32, K, Kp);
    const int m = std::max(1, o.check_every);
    const bool bf16 = in.prec == L0L2_BF16;
    // the BF16 split form's floor is about 1e-4; single-term blocks are anchored
    // on the FP32 state, whose floor is the FP32 one
    const double switch_tol = (bf16 && !bf16_single(ctx, Kp) ? 200.0 : 50.0) * o.tol_node;
    bool fp64 = false;
    if (in.prec == L0L2_FP8) {
        // FP8 storage: anchored sweeps from the start, on the FP64 state
        hipLaunchKernelGGL(k_promote, dim3(grid1d(Kp * in.ldp)), dim3(256), 0, ctx->stream, s32.beta, s32.V, s64.beta,
                           s64.V, s64.W, s64.c, in.mp.rho, in.ldp, Kp * in.ldp);
        HIPCHK(hipGetLastError());
        fp64 = true;
    }
    int cnt[3], best_above = 1 << 30, flat = 0;
    int64_t active = K;
    // single-term blocks before the switch run two check intervals per block:
    // their gap sits above the FP32 floor, so the checks mostly steer the
    // switch, and each block's first sweep is the split-form one that renews
    // the anchor
    const bool long_blocks = bf16 && bf16_single(ctx, Kp);
    for (int t = 0; t < o.max_iter;) {
        check_cancel(ctx);
        const int n = std::min(!fp64 && long_blocks ? 2 * m : m, o.max_iter - t);
        const int kind = fp64 ? SK_ANCH : (bf16 ? SK_BF16 : SK_F32);
        run_block(ctx, kind, Kp, n, o.tol_node, switch_tol, active, t + n >= o.max_iter, cnt);
        t += n;
        active = cnt[0];
        if (cnt[0] == 0) break;
        if (!fp64) {
            if (cnt[1] < best_above) { best_above = cnt[1]; flat = 0; }
            else ++flat;
            if (cnt[1] == 0 || flat >= 5 || 2 * t >= o.max_iter) {
                hipLaunchKernelGGL(k_promote, dim3(grid1d(Kp * in.ldp)), dim3(256), 0, ctx->stream, s32.beta, s32.V,
                                   s64.beta, s64.V, s64.W, s64.c, in.mp.rho, in.ldp, Kp * in.ldp);
                HIPCHK(hipGetLastError());
                fp64 = true;
            }
        }
    }
    if (fp64) {
        hipLaunchKernelGGL(k_demote, dim3(grid1d(Kp * in.ldp)), dim3(256), 0, ctx->stream, s64.beta, s64.V, s32.beta,
                           s32.V, Kp * in.ldp);
        HIPCHK(hipGetLastError());
    }
}

// Continuous batching of node relaxations (the batching pattern's slot
// refill): N queued nodes run through the K slots of the workspace; at each
// block boundary the slots whose nodes retired (converged, or at their own
// sweep budget) hand their results to the nodes' queue positions and take the
// next queued nodes, so the sweeps keep covering a full batch until the queue
// runs dry.  Each node has its own sweep count and budget.  FP64 mode runs its
// plain sweeps; the reduced modes run anchored from the first sweep (FP64
// state, an FP64 anchor per block, the reduced products act on the movement
// since it), so a node that joins a running batch needs no phase of its own.
template <class T>
void solve_queue_t(l0l2_ctx *ctx, int N, const uint8_t *qcodes, void *qbeta, void *qv, int K,
                   const l0l2_admm_opts &o, double *qlb, double *qprimal, int32_t *qiters, int32_t *qstatus) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    const int64_t Kp = round_up(K, kPadNodes), ldp = in.ldp;
    const bool fp64 = in.prec == L0L2_FP64;
    if (!fp64) decide_form(ctx, Kp);
    Sweep<double> s64 = sweep64(ctx);
    Sweep<float> s32 = sweep32(ctx);
    const T *c = fp64 ? (const T *)s64.c : (const T *)s32.c;
    T *beta = fp64 ? (T *)s64.beta : (T *)s32.beta;
    T *V = fp64 ? (T *)s64.V : (T *)s32.V;
    T *W = fp64 ? (T *)s64.W : (T *)s32.W;
    hipLaunchKernelGGL(k_set_active, dim3((unsigned)((Kp + 255) / 256)), dim3(256), 0, s, ws.active.as<int>(),
                       ws.status.as<int>(), ws.iters.as<int>(), ws.list.as<int>(), ws.clist.as<int>(), (int64_t)0,
                       Kp, ws.sweep_no.as<int>(), ws.start.as<int>());
    HIPCHK(hipGetLastError());
    std::vector<int> slot_q((size_t)Kp, -1), freed, pairs, dl;
    DevBuf dpairs;
    dpairs.ensure(sizeof(int) * 2 * (size_t)Kp);
    int next = 0;
    int64_t active = 0;
    // slots `freed` take the next queued nodes (as many as remain)
    auto refill = [&](std::vector<int> &slots) {
        const int m = (int)std::min<int64_t>((int64_t)slots.size(), (int64_t)N - next);
        if (m <= 0) return;
        pairs.assign((size_t)2 * m, 0);
        for (int e = 0; e < m; ++e) {
            pairs[(size_t)2 * e] = slots[(size_t)e];
            pairs[(size_t)2 * e + 1] = next;
            slot_q[(size_t)slots[(size_t)e]] = next++;
        }
        HIPCHK(hipMemcpyAsync(dpairs.ptr, pairs.data(), sizeof(int) * 2 * m, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL((k_queue_load<T>), dim3((unsigned)((ldp + 255) / 256), (unsigned)m), dim3(256), 0, s,
                           qcodes, (const T *)qbeta, (const T *)qv, in.p, dpairs.as<int>(), ws.codes.as<uint8_t>(),
                           beta, V, W, c, (T)in.mp.rho, s64.beta, s64.V, s64.W, (const double *)s64.c, in.mp.rho,
                           fp64 ? 0 : 1, ldp, ws.active.as<int>(), ws.status.as<int>(), ws.iters.as<int>(),
                           ws.start.as<int>(), (const int *)ws.sweep_no.ptr);
        hipLaunchKernelGGL(k_list_append, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, ws.list.as<int>(),
                           active, (const int *)dpairs.ptr, m);
        HIPCHK(hipGetLastError());
        // the pairs buffer is reused by the next refill only after a block has synchronised
        active += m;
    };
    freed.clear();
    for (int k = 0; k < (int)std::min<int64_t>(K, N); ++k) freed.push_back(k);
    refill(freed);
    const int m = std::max(1, o.check_every);
    const int kind = fp64 ? SK_F64 : SK_ANCH;
    int cnt[3];
    while (active > 0) {
        check_cancel(ctx);
        run_block(ctx, kind, Kp, m, o.tol_node, o.tol_node, active, false, cnt, o.max_iter);
        active = cnt[0];
        const int nd = cnt[2];
        if (nd <= 0) continue;
        dl.assign((size_t)nd, 0);
        HIPCHK(hipMemcpyAsync(dl.data(), ws.dlist.ptr, sizeof(int) * nd, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        pairs.assign((size_t)2 * nd, 0);
        for (int e = 0; e < nd; ++e) {
            pairs[(size_t)2 * e] = dl[(size_t)e];
            pairs[(size_t)2 * e + 1] = slot_q[(size_t)dl[(size_t)e]];
            slot_q[(size_t)dl[(size_t)e]] = -1;
        }
        HIPCHK(hipMemcpyAsync(dpairs.ptr, pairs.data(), sizeof(int) * 2 * nd, hipMemcpyHostToDevice, s));
        const dim3 gs((unsigned)((in.p + 255) / 256), (unsigned)nd);
        if (fp64)
            hipLaunchKernelGGL((k_queue_store<double, double>), gs, dim3(256), 0, s, (const int *)dpairs.ptr,
                               (const double *)s64.beta, (const double *)s64.V, ldp, in.p, (const double *)ws.lb.ptr,
                               (const double *)ws.primal.ptr, (const int *)ws.iters.ptr, (const int *)ws.status.ptr,
                               (double *)qbeta, (double *)qv, qlb, qprimal, qiters, qstatus);
        else
            hipLaunchKernelGGL((k_queue_store<double, float>), gs, dim3(256), 0, s, (const int *)dpairs.ptr,
                               (const double *)s64.beta, (const double *)s64.V, ldp, in.p, (const double *)ws.lb.ptr,
                               (const double *)ws.primal.ptr, (const int *)ws.iters.ptr, (const int *)ws.status.ptr,
                               (float *)qbeta, (float *)qv, qlb, qprimal, qiters, qstatus);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));   // the pairs buffer is rewritten by the refill below
        freed.assign(dl.begin(), dl.end());
        refill(freed);
    }
}

template <class T>
void sweeps_t(l0l2_ctx *ctx, const Sweep<T> &sw, int K, int sweeps) {
    const int64_t Kp = round_up(K, kPadNodes);
    init_batch<T>(ctx, sw, K, Kp);
    for (int t = 1; t <= sweeps; ++t) sweep_once<T>(ctx, sw, Kp, t == sweeps, K);
}

}  // namespace

void run_queue(l0l2_ctx *ctx, int N, const uint8_t *codes, void *beta, void *v, int K, const l0l2_admm_opts &o,
               double *lb, double *primal, int32_t *iters, int32_t *status) {
    Workspace &ws = ctx->ws;
    ws.stat_blocks = ws.stat_sparse = ws.stat_node_blocks = 0;
    if (ctx->inst.prec == L0L2_FP64) solve_queue_t<double>(ctx, N, codes, beta, v, K, o, lb, primal, iters, status);
    else solve_queue_t<float>(ctx, N, codes, beta, v, K, o, lb, primal, iters, status);
}

void ensure_workspace(l0l2_ctx *ctx, int64_t K) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    const int64_t Kp = round_up(std::max<int64_t>(K, 1), kPadNodes);
    if (Kp <= ws.cap && ws.host_counter) return;
    const size_t sb = state_bytes(in.prec);
    const int64_t np = in.np, pp = in.pp, ldp = in.ldp;
    ws.W.ensure(sb * Kp * ldp);
    ws.beta.ensure(sb * Kp * ldp);
    ws.V.ensure(sb * Kp * ldp);
    ws.B.ensure(sb * Kp * ldp);
    ws.U.ensure(sb * Kp * in.ldu);
    ws.R.ensure(8 * Kp * in.ldu64);
    ws.codes.ensure((size_t)(Kp * ldp));
    ws.rpart.ensure(8 * 4 * Kp * (np / 32));
    ws.part.ensure(8 * 3 * Kp * (pp / 32));
    ws.gpart.ensure(8 * 5 * Kp * (pp / 16));
    ws.gate.ensure(sizeof(int));
    ws.needs.ensure(4 * Kp);
    ws.gest.ensure(8 * Kp);
    ws.clist.ensure(4 * Kp);
    ws.list.ensure(4 * Kp);
    ws.nlist.ensure(4 * Kp);
    ws.ncount.ensure(sizeof(int));
    ws.active.ensure(4 * Kp);
    ws.iters.ensure(4 * Kp);
    ws.status.ensure(4 * Kp);
    ws.lb.ensure(8 * Kp);
    ws.primal.ensure(8 * Kp);
    ws.counter.ensure(3 * sizeof(int));
    ws.start.ensure(4 * Kp);
    ws.dlist.ensure(4 * Kp);
    ws.sweep_no.ensure(sizeof(int));
    drop_graphs(ctx);
    ++ws.gen;
    if (!ws.host_counter) HIPCHK(hipHostMalloc((void **)&ws.host_counter, 3 * sizeof(int), hipHostMallocDefault));
    if (in.prec != L0L2_FP64) {
        ws.W2.ensure(4 * Kp * ldp);
        HIPCHK(hipMemsetAsync(ws.W2.ptr, 0, 4 * Kp * ldp, ctx->stream));
        ws.Wa.ensure(8 * Kp * ldp);
        ws.Za.ensure(8 * Kp * ldp);
        ws.W64.ensure(8 * Kp * ldp);
        ws.beta64.ensure(8 * Kp * ldp);
        ws.V64.ensure(8 * Kp * ldp);
        ws.B64.ensure(8 * Kp * ldp);
        ws.U64.ensure(8 * Kp * in.ldu64);
        HIPCHK(hipMemsetAsync(ws.B64.ptr, 0, 8 * Kp * ldp, ctx->stream));
    }
    if (in.prec == L0L2_BF16) {
        ws.Wa32.ensure(4 * Kp * ldp);
        ws.Za32.ensure(4 * Kp * ldp);
        for (int i = 0; i < 2; ++i) {
            ws.Dbf[i].ensure(2 * Kp * ldp);
            HIPCHK(hipMemsetAsync(ws.Dbf[i].ptr, 0, 2 * Kp * ldp, ctx->stream));
        }
    }
    // inactive padded rows must read as zeros on first use
    HIPCHK(hipMemsetAsync(ws.W.ptr, 0, sb * Kp * ldp, ctx->stream));
    HIPCHK(hipMemsetAsync(ws.B.ptr, 0, sb * Kp * ldp, ctx->stream));
    ws.cap = Kp;
}

void load_batch(l0l2_ctx *ctx, int K, const uint8_t *codes, const void *beta, const void *v, bool codes_on_host) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    ensure_workspace(ctx, K);
    const int64_t Kp = round_up(K, kPadNodes);
    const uint8_t *dcodes = codes;
    DevBuf tmp;
    if (codes_on_host) {
        tmp.ensure((size_t)K * in.p);
        HIPCHK(hipMemcpyAsync(tmp.ptr, codes, (size_t)K * in.p, hipMemcpyHostToDevice, s));
        dcodes = tmp.as<uint8_t>();
    }
    const int64_t ldp = in.ldp;
    hipLaunchKernelGGL(k_load_codes, dim3(grid1d(Kp * ldp)), dim3(256), 0, s, dcodes, (int64_t)K, in.p,
                       ws.codes.as<uint8_t>(), Kp, ldp);
    if (in.prec == L0L2_FP64) {
        hipLaunchKernelGGL(k_load_state<double>, dim3(grid1d(Kp * ldp)), dim3(256), 0, s, (const double *)beta,
                           (int64_t)K, in.p, ws.beta.as<double>(), Kp, ldp);
        hipLaunchKernelGGL(k_load_state<double>, dim3(grid1d(Kp * ldp)), dim3(256), 0, s, (const double *)v,
                           (int64_t)K, in.p, ws.V.as<double>(), Kp, ldp);
    } else {
        hipLaunchKernelGGL(k_load_state<float>, dim3(grid1d(Kp * ldp)), dim3(256), 0, s, (const float *)beta,
                           (int64_t)K, in.p, ws.beta.as<float>(), Kp, ldp);
        hipLaunchKernelGGL(k_load_state<float>, dim3(grid1d(Kp * ldp)), dim3(256), 0, s, (const float *)v,
                           (int64_t)K, in.p, ws.V.as<float>(), Kp, ldp);
    }
    HIPCHK(hipGetLastError());
    if (codes_on_host) HIPCHK(hipStreamSynchronize(s));
}

void store_batch(l0l2_ctx *ctx, int K, void *beta, void *v, void *b) {
    Instance &in = ctx->inst;
    Workspace &ws = ctx->ws;
    hipStream_t s = ctx->stream;
    unsigned g = grid1d((int64_t)K * in.p);
    if (in.prec == L0L2_FP64) {
        if (beta) hipLaunchKernelGGL(k_store_state<double>, dim3(g), dim3(256), 0, s, ws.beta.as<double>(), (int64_t)K, in.p, in.ldp, (double *)beta);
        if (v) hipLaunchKernelGGL(k_store_state<double>, dim3(g), dim3(256), 0, s, ws.V.as<double>(), (int64_t)K, in.p, in.ldp, (double *)v);
        if (b) hipLaunchKernelGGL(k_store_state<double>, dim3(g), dim3(256), 0, s, ws.B.as<double>(), (int64_t)K, in.p, in.ldp, (double *)b);
    } else {
        if (beta) hipLaunchKernelGGL(k_store_state<float>, dim3(g), dim3(256), 0, s, ws.beta.as<float>(), (int64_t)K, in.p, in.ldp, (float *)beta);
        if (v) hipLaunchKernelGGL(k_store_state<float>, dim3(g), dim3(256), 0, s, ws.V.as<float>(), (int64_t)K, in.p, in.ldp, (float *)v);
        if (b) hipLaunchKernelGGL(k_store_state<float>, dim3(g), dim3(256), 0, s, ws.B.as<float>(), (int64_t)K, in.p, in.ldp, (float *)b);
    }
    HIPCHK(hipGetLastError());
}

void run_sweeps(l0l2_ctx *ctx, int K, int sweeps, bool) {
    if (ctx->inst.prec == L0L2_FP8) fail(L0L2_E_UNSUPPORTED, "FP8 storage runs anchored solves only");
    if (ctx->inst.prec == L0L2_FP64) {
        sweeps_t<double>(ctx, sweep64(ctx), K, sweeps);
    } else if (ctx->inst.prec == L0L2_FP32) {
        sweeps_t<float>(ctx, sweep32(ctx), K, sweeps);
    } else {
        const int64_t Kp = round_up(K, kPadNodes);
        Sweep<float> s32 = sweep32(ctx);
        init_batch<float>(ctx, s32, K, Kp);
        for (int t = 1; t <= sweeps; ++t) sweep_once_bf16(ctx, Kp, t == sweeps, K, false, false);
    }
}

void run_solve(l0l2_ctx *ctx, int K, const l0l2_admm_opts &o) {
    ctx->ws.stat_blocks = ctx->ws.stat_sparse = ctx->ws.stat_node_blocks = 0;
    if (ctx->inst.prec == L0L2_FP64) solve_plain<double>(ctx, sweep64(ctx), K, o);
    else solve_mixed(ctx, K, o);
}

// The batch axis of the autotuner.  Each candidate K (32, 64, ... up to k_max)
// solves a batch of K nodes with every coordinate free from a cold start, for
// two blocks of the default check interval with a zero tolerance (no node
// retires, so every node does every sweep): the precision path, gap checks,
// live buckets and graph replay of a real solve.  The first solve settles the
// tile shapes and graphs of that K, the second is timed on the host clock.  The
// chosen K is the smallest whose node-sweeps per second reach frac of the best
// candidate's: past it a larger batch adds little throughput, while in a
// best-first tree it solves nodes that a better incumbent found meanwhile would
// have pruned.
int tune_batch_size(l0l2_ctx *ctx, int k_max, double frac, std::vector<double> &rates) {
    Instance &in = ctx->inst;
    const size_t sb = state_bytes(in.prec);
    rates.clear();
    l0l2_admm_opts o{};
    o.tol_node = 0.0;
    o.check_every = 10;
    o.max_iter = 2 * o.check_every;
    DevBuf codes, beta, v;
    int best_k = kPadNodes;
    double best = 0.0;
    for (int K = kPadNodes; K <= k_max; K *= 2) {
        codes.ensure((size_t)K * in.p);
        beta.ensure(sb * K * in.p);
        v.ensure(sb * K * in.p);
        double secs = 0.0;
        for (int rep = 0; rep < 2; ++rep) {
            HIPCHK(hipMemsetAsync(codes.ptr, 0, (size_t)K * in.p, ctx->stream));   // every coordinate free
            HIPCHK(hipMemsetAsync(beta.ptr, 0, sb * K * in.p, ctx->stream));
            HIPCHK(hipMemsetAsync(v.ptr, 0, sb * K * in.p, ctx->stream));
            load_batch(ctx, K, codes.as<uint8_t>(), beta.ptr, v.ptr, false);
            HIPCHK(hipStreamSynchronize(ctx->stream));
            const auto t0 = std::chrono::steady_clock::now();
            run_solve(ctx, K, o);
            HIPCHK(hipStreamSynchronize(ctx->stream));
            secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        const double r = (double)K * o.max_iter / std::max(secs, 1e-9);
        rates.push_back(r);
        best = std::max(best, r);
    }
    for (size_t i = 0; i < rates.size(); ++i)
        if (rates[i] >= frac * best) {
            best_k = kPadNodes << i;
            break;
        }
    in.tuned_K = best_k;
    return best_k;
}

// Bound at b already loaded in ws.B (codes in ws.codes): fills ws.lb.
void run_dual_bound(l0l2_ctx *ctx, int K, const void *) {
    const int64_t Kp = round_up(K, kPadNodes);
    Workspace &ws = ctx->ws;
    hipLaunchKernelGGL(k_set_active, dim3((unsigned)((Kp + 255) / 256)), dim3(256), 0, ctx->stream,
                       ws.active.as<int>(), ws.status.as<int>(), ws.iters.as<int>(), ws.list.as<int>(),
                       ws.clist.as<int>(), (int64_t)K, Kp, ws.sweep_no.as<int>(), ws.start.as<int>());
    if (ctx->inst.prec == L0L2_FP64)
        check_once<double>(ctx, ws.B.as<double>(), ws.B.as<double>(), Kp, 0.0, 0.0, 1);
    else
        check_once<float>(ctx, ws.B.as<float>(), ws.B.as<float>(), Kp, 0.0, 0.0, 1);
}

int bupdate_form(l0l2_ctx *ctx, double ms[2]) {
    ms[0] = ctx->inst.form_ms[0];
    ms[1] = ctx->inst.form_ms[1];
    return gram_form(ctx) ? 2 : 1;
}

}  // namespace l0l2
