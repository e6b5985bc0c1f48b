// Matching-pursuit root heuristic (Sec. 3.5; the forward and backward score
// closed forms of App. A.2), FP64 with the original X.
//
// From the empty support, a forward step adds the coordinate outside S whose
// single-coordinate move lowers F(S, beta) = 1/2 ||y - X beta||^2 +
// lambda2 ||beta||^2 + lambda0 |S| the most (the other coordinates frozen):
//   c_j = X_j^T r, D_j = ||X_j||^2 + 2 lambda2, b_j = clip(c_j / D_j, -M, M),
//   Delta_j = -b_j c_j + D_j b_j^2 / 2 + lambda0,
// taken when Delta_j < 0; a backward step removes the coordinate of S whose
// removal lowers F the most:
//   Delta_j = beta_j c_j + (||X_j||^2 / 2 - lambda2) beta_j^2 - lambda0.
// Steps alternate forward / backward; the run ends when a forward step and the
// backward step after it both find no improving move, or after max_moves moves.
// Ties go to the smallest index.
//
// Each step is two launches: the scores (one wave per column: c_j and ||X_j||^2
// from one pass over the column, then Delta_j, and a per-workgroup minimum over
// the candidates of the step's kind) and the move (one workgroup: the minimum
// over the workgroups, then the exact update of beta, S and r = y - X beta).
// The loop state (step kind, moves made, end flag) lives on the device, so the
// host queues steps in groups and reads the end flag once per group.
#include <cmath>
#include <vector>

#include "device_math.hpp"
#include "internal.hpp"

namespace l0l2 {

namespace {

constexpr int kMpWaves = 4;   // columns per scoring workgroup
constexpr int kMpGroup = 32;  // steps queued between reads of the end flag

struct MpState {
    int done;      // no further move
    int nmoves;    // moves made
    int moved;     // a move in the current forward / backward round
    int step;      // steps taken (even: forward, odd: backward)
    double delta;  // score of the last move
};

struct MpArgs {
    int64_t n, p, ldx;
    double l0, l2, M;
    int max_moves;
};

__global__ void k_mp_init(const double *__restrict__ y, double *__restrict__ r, double *__restrict__ beta,
                          uint8_t *__restrict__ mask, MpState *st, int64_t np, int64_t pp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) r[i] = y[i];
    if (i < pp) {
        beta[i] = 0.0;
        mask[i] = 0;
    }
    if (i == 0) *st = MpState{0, 0, 0, 0, 0.0};
}

// Scores of the current step's candidates; writes the workgroup's smallest
// negative score and its column (+inf / -1 when it has none).
__global__ __launch_bounds__(64 * kMpWaves) void k_mp_scores(const double *__restrict__ X, const double *__restrict__ r,
                                                             const double *__restrict__ beta,
                                                             const uint8_t *__restrict__ mask,
                                                             double *__restrict__ bnew, double *__restrict__ pdelta,
                                                             int *__restrict__ pidx, const MpState *st, MpArgs a) {
    if (st->done) return;
    const int want = st->step & 1;   // 0: forward (j outside S), 1: backward (j in S)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * kMpWaves + w;
    double best = INFINITY;
    if (j < a.p) {
        const double *col = X + j * a.ldx;
        double c = 0.0, q = 0.0;
        for (int64_t i = lane; i < a.n; i += 64) {
            const double x = col[i];
            c = fma(x, r[i], c);
            q = fma(x, x, q);
        }
        for (int off = 32; off > 0; off >>= 1) {
            c += __shfl_xor(c, off);
            q += __shfl_xor(q, off);
        }
        const int in_s = mask[j] != 0;
        double d;
        if (in_s) {
            const double b = beta[j];
            d = b * c + (0.5 * q - a.l2) * b * b - a.l0;
        } else {
            const double D = q + 2.0 * a.l2;
            const double b = clip_box(c / D, a.M);
            d = -b * c + 0.5 * D * b * b + a.l0;
            if (lane == 0) bnew[j] = b;
        }
        if (in_s == want && d < 0.0) best = d;
    }
    __shared__ double sd[kMpWaves];
    __shared__ int64_t sj[kMpWaves];
    if (lane == 0) {
        sd[w] = best;
        sj[w] = best < INFINITY ? j : -1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bd = INFINITY;
        int64_t bj = -1;
        for (int u = 0; u < kMpWaves; ++u)   // columns in increasing order: strict < keeps the smallest index
            if (sj[u] >= 0 && sd[u] < bd) {
                bd = sd[u];
                bj = sj[u];
            }
        pdelta[blockIdx.x] = bd;
        pidx[blockIdx.x] = (int)bj;
    }
}

// The step's move: the smallest score over the workgroups (ties: smallest
// column), then beta, S and r updated exactly as the move defines them.
__global__ __launch_bounds__(256) void k_mp_move(const double *__restrict__ X, double *__restrict__ r,
                                                 double *__restrict__ beta, uint8_t *__restrict__ mask,
                                                 const double *__restrict__ bnew, const double *__restrict__ pdelta,
                                                 const int *__restrict__ pidx, int nparts, int32_t *__restrict__ moves,
                                                 MpState *st, MpArgs a) {
    if (st->done) return;
    __shared__ double sd[256];
    __shared__ int si[256];
    const int tid = threadIdx.x;
    double bd = INFINITY;
    int bj = -1;
    for (int e = tid; e < nparts; e += 256) {
        const int j = pidx[e];
        const double d = pdelta[e];
        if (j >= 0 && (d < bd || (d == bd && j < bj))) {
            bd = d;
            bj = j;
        }
    }
    sd[tid] = bd;
    si[tid] = bj;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) {
            const int o = tid + s;
            if (si[o] >= 0 && (si[tid] < 0 || sd[o] < sd[tid] || (sd[o] == sd[tid] && si[o] < si[tid]))) {
                sd[tid] = sd[o];
                si[tid] = si[o];
            }
        }
        __syncthreads();
    }
    const int j = si[0];
    const int want = st->step & 1;
    if (j >= 0) {
        // forward: r <- r - X_j b; backward: r <- r + X_j beta_j (products rounded
        // before the update, as the move's definition reads)
        const double b = want ? -beta[j] : bnew[j];
        const double *col = X + (int64_t)j * a.ldx;
        for (int64_t i = tid; i < a.n; i += 256) r[i] = __dsub_rn(r[i], __dmul_rn(col[i], b));
        __syncthreads();
        if (tid == 0) {
            beta[j] = want ? 0.0 : b;
            mask[j] = want ? 0 : 1;
            moves[st->nmoves] = want ? -(j + 1) : j + 1;
            st->nmoves += 1;
            st->moved = 1;
            st->delta = sd[0];
        }
    }
    if (tid == 0) {
        if (want) {
            // end of a forward / backward round
            if (!st->moved) st->done = 1;
            st->moved = 0;
        }
        st->step += 1;
        if (st->nmoves >= a.max_moves) st->done = 1;
    }
}

}  // namespace

void run_matching_pursuit(l0l2_ctx *ctx, int max_moves, uint8_t *mask_host, double *beta_host, int32_t *moves_host,
                          int32_t *n_moves, double *obj) {
    Instance &in = ctx->inst;
    hipStream_t s = ctx->stream;
    const int64_t np = in.np, pp = in.pp, n = in.n, p = in.p;
    const int nparts = (int)((p + kMpWaves - 1) / kMpWaves);
    DevBuf r, beta, mask, bnew, pdelta, pidx, moves, stb;
    r.ensure(sizeof(double) * np);
    beta.ensure(sizeof(double) * pp);
    mask.ensure(pp);
    bnew.ensure(sizeof(double) * pp);
    pdelta.ensure(sizeof(double) * nparts);
    pidx.ensure(sizeof(int) * nparts);
    moves.ensure(sizeof(int32_t) * (size_t)std::max(max_moves, 1));
    stb.ensure(sizeof(MpState));
    MpState *st = stb.as<MpState>();
    const MpArgs a{n, p, in.ldx, in.mp.l0, in.mp.l2, in.mp.M, max_moves};
    const int64_t ninit = std::max(np, pp);
    hipLaunchKernelGGL(k_mp_init, dim3((unsigned)((ninit + 255) / 256)), dim3(256), 0, s, in.y64.as<double>(),
                       r.as<double>(), beta.as<double>(), mask.as<uint8_t>(), st, np, pp);
    HIPCHK(hipGetLastError());
    MpState hs{};
    // every round of two steps either moves or ends the run, so at most
    // 2 (max_moves + 1) steps are needed
    const int64_t max_steps = 2 * ((int64_t)max_moves + 1);
    for (int64_t done_steps = 0; done_steps < max_steps; done_steps += kMpGroup) {
        check_cancel(ctx);
        for (int g = 0; g < kMpGroup; ++g) {
            hipLaunchKernelGGL(k_mp_scores, dim3((unsigned)nparts), dim3(64 * kMpWaves), 0, s, in.X64.as<double>(),
                               (const double *)r.ptr, (const double *)beta.ptr, (const uint8_t *)mask.ptr,
                               bnew.as<double>(), pdelta.as<double>(), pidx.as<int>(), (const MpState *)st, a);
            hipLaunchKernelGGL(k_mp_move, dim3(1), dim3(256), 0, s, in.X64.as<double>(), r.as<double>(),
                               beta.as<double>(), mask.as<uint8_t>(), (const double *)bnew.ptr,
                               (const double *)pdelta.ptr, (const int *)pidx.ptr, nparts, moves.as<int32_t>(), st, a);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&hs, st, sizeof(MpState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hs.done) break;
    }
    std::vector<double> rh((size_t)n);
    HIPCHK(hipMemcpyAsync(rh.data(), r.ptr, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(beta_host, beta.ptr, sizeof(double) * p, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(mask_host, mask.ptr, (size_t)p, hipMemcpyDeviceToHost, s));
    if (moves_host && hs.nmoves > 0)
        HIPCHK(hipMemcpyAsync(moves_host, moves.ptr, sizeof(int32_t) * hs.nmoves, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *n_moves = hs.nmoves;
    // F(S, beta) at the heuristic's coefficients, from its residual
    double rr = 0.0, bb = 0.0;
    int64_t ns = 0;
    for (int64_t i = 0; i < n; ++i) rr += rh[(size_t)i] * rh[(size_t)i];
    for (int64_t j = 0; j < p; ++j) {
        bb += beta_host[j] * beta_host[j];
        ns += mask_host[j] != 0;
    }
    *obj = 0.5 * rr + in.mp.l2 * bb + in.mp.l0 * (double)ns;
}

}  // namespace l0l2
