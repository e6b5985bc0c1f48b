// Rounding, branching and incumbent refinement (Sec. 3.3 and 3.4), FP64.
#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>
#include <vector>

#include "device_math.hpp"
#include "internal.hpp"

// Residual scratch of the allocation-free refinement (one row of the padded n
// doubles per node), a file-scope device array: every device the library runs
// on holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address); it uses the per-device address that hipGetSymbolAddress returns.
static __device__ __align__(256) double scratch[l0l2::kNoAllocScratchBytes / sizeof(double)];

namespace l0l2 {

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoAllocMaxDevices] = {};

}  // namespace

void *noalloc_scratch(int device) {
    if (device < 0 || device >= kNoAllocMaxDevices)
        fail(L0L2_E_UNSUPPORTED, "the allocation-free entry points support device indices below " +
                                     std::to_string(kNoAllocMaxDevices));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        // the caller has made `device` current
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            fail(L0L2_E_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        }
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

namespace {

constexpr int kSMax = 1024;   // largest support refined by one workgroup

// Deterministic block sum broadcast to every thread (256 threads).
__device__ __forceinline__ double bsum(double v, double *sh) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

__device__ __forceinline__ double bmax(double v, double *sh) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

struct RoundArgs {
    double s, M;
    int free_quad;
    int64_t p;
};

// One workgroup per node.  S = F1 u {free j : z_j >= 1/2}; branching index =
// the free j of largest floor(2^20 min(z_j, 1 - z_j)), ties to the smallest j;
// if that score is 0 for every free j, the free j of largest |beta_j|.
template <class T>
__global__ __launch_bounds__(256) void k_round_branch(const uint8_t *__restrict__ codes, int64_t ldc,
                                                      const T *__restrict__ beta, int64_t ldb,
                                                      uint8_t *__restrict__ support, int32_t *__restrict__ ssize,
                                                      int32_t *__restrict__ bj, int32_t *__restrict__ zup,
                                                      int32_t *__restrict__ nfree, RoundArgs ra) {
    __shared__ double shs[256];
    __shared__ int64_t shj[256];
    __shared__ double sha[256];
    __shared__ int64_t shja[256];
    __shared__ int shc[256], shf[256];
    const int64_t k = blockIdx.x;
    const int tid = threadIdx.x;
    double bsc = -1.0, babs = -1.0;
    int64_t bjj = INT64_MAX, bja = INT64_MAX;
    int cnt = 0, nf = 0;
    for (int64_t j = tid; j < ra.p; j += 256) {
        uint8_t code = codes[k * ldc + j];
        double b = (double)beta[k * ldb + j];
        double z = z_of(b, code, ra.s, ra.M, ra.free_quad);
        uint8_t sup = (code == CODE_FIX1) || (code == CODE_FREE && z >= 0.5);
        support[k * ra.p + j] = sup;
        cnt += sup;
        if (code == CODE_FREE) {
            ++nf;
            double f = z < 1.0 - z ? z : 1.0 - z;
            double sc = floor(f * 1048576.0);
            if (sc > bsc) { bsc = sc; bjj = j; }
            double ab = fabs(b);
            if (ab > babs) { babs = ab; bja = j; }
        }
    }
    shs[tid] = bsc; shj[tid] = bjj; sha[tid] = babs; shja[tid] = bja; shc[tid] = cnt; shf[tid] = nf;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) {
            int o = tid + st;
            if (shs[o] > shs[tid] || (shs[o] == shs[tid] && shj[o] < shj[tid])) { shs[tid] = shs[o]; shj[tid] = shj[o]; }
            if (sha[o] > sha[tid] || (sha[o] == sha[tid] && shja[o] < shja[tid])) { sha[tid] = sha[o]; shja[tid] = shja[o]; }
            shc[tid] += shc[o];
            shf[tid] += shf[o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        ssize[k] = shc[0];
        nfree[k] = shf[0];
        int64_t j = -1;
        if (shf[0] > 0) j = shs[0] <= 0.0 ? shja[0] : shj[0];
        bj[k] = (int32_t)j;
        int up = 0;
        if (j >= 0) up = z_of((double)beta[k * ldb + j], CODE_FREE, ra.s, ra.M, ra.free_quad) >= 0.5;
        zup[k] = up;
    }
}

struct FistaArgs {
    double l0, l2, M, tol;
    int max_iter;
    int64_t n, np, p;
    int64_t ldx;   // column stride of X
};

// U_S(v) = 1/2 ||X_S v - y||^2 + l2 ||v||^2; optionally keeps the residual.
__device__ double U_S(const double *__restrict__ X, int64_t ldx, const double *__restrict__ y, const int *idx, int k,
                      const double *v, double *res, bool keep, double *sh, const FistaArgs &fa) {
    double rr = 0.0;
    for (int64_t i = threadIdx.x; i < fa.n; i += 256) {
        double s = 0.0;
        for (int a = 0; a < k; ++a) s += X[(int64_t)idx[a] * ldx + i] * v[a];
        double r = s - y[i];
        if (keep) res[i] = r;
        rr += r * r;
    }
    double bb = 0.0;
    for (int a = threadIdx.x; a < k; a += 256) bb += v[a] * v[a];
    rr = bsum(rr, sh);
    bb = bsum(bb, sh);
    return 0.5 * rr + fa.l2 * bb;
}

// Fast proximal gradient on each support (eqs. fpg_extrapolate .. fpg_armijo),
// one workgroup of 4 waves per node.  Start at the node iterate on S; alpha_0 =
// 4 / (||X_S||_F^2 + 2 l2), halved on each Armijo failure (at most 60 times per
// iteration) and carried over; stop on |dU| <= tol max(1, U) or max|d beta| <=
// 1e-10; at most max_iter iterations.
//
// Supports of up to kGramMax = 64 coordinates build G = X_S^T X_S once with FP64
// MFMA (the 4 waves split the rows of X_S, lower block triangle only) and keep it
// in LDS with g = X_S^T y; one wave then runs the iterations with coordinate a
// on lane a: U(b) = 1/2 ||y||^2 - g^T b + 1/2 b^T G b + l2 ||b||^2 and
// grad = G b - g + 2 l2 b, every sum a wave reduction (no workgroup barrier).
// Larger supports stream X_S once per evaluation with all 4 waves.  Either way
// the returned objective F(S, beta) is evaluated from the residual y - X_S beta
// in FP64.
constexpr int kGramMax = 64;

struct FistaShared {
    int idx[kSMax];
    double cur[kSMax], prev[kSMax], ext[kSMax], nxt[kSMax], grad[kSMax];
    double G[kGramMax * kGramMax];   // column-major, leading dimension kGramMax
    double vb[kGramMax];
    double sh[4];
    int shw[4];
    int it;
};

// Wave-wide reductions of doubles without the LDS crossbar: DPP row
// butterflies (xor 1 and xor 2 within quads, then the half-row and row mirrors)
// leave every lane of a 16-lane row with the row's value, and the four row
// values are read from lanes 0, 16, 32 and 48 and combined in the same order on
// every lane, so all lanes return identical bits.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

// Sum over the 64 lanes of a wave; every lane receives the same value.
__device__ __forceinline__ double wsum(double v) {
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    v += dpp_f64<kDppHalfMirror>(v);
    v += dpp_f64<kDppMirror>(v);
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Maximum over the 64 lanes of a wave; every lane receives the same value.
__device__ __forceinline__ double wmax(double v) {
    v = fmax(v, dpp_f64<kDppXor1>(v));
    v = fmax(v, dpp_f64<kDppXor2>(v));
    v = fmax(v, dpp_f64<kDppHalfMirror>(v));
    v = fmax(v, dpp_f64<kDppMirror>(v));
    return fmax(fmax(lane_f64(v, 0), lane_f64(v, 16)), fmax(lane_f64(v, 32), lane_f64(v, 48)));
}

// Lane a < k: (G v)_a for v held one coordinate per lane (wave-local LDS
// broadcast through sm.vb); returns the lane's share of U(v) - yy/2 in *part.
__device__ __forceinline__ double gram_mv(FistaShared &sm, double v, int k, int lane) {
    __builtin_amdgcn_wave_barrier();
    sm.vb[lane] = v;
    __builtin_amdgcn_wave_barrier();
    double s = 0.0;
    if (lane < k) {
        // four independent partial sums keep several LDS reads in flight
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int b = 0;
        for (; b + 4 <= k; b += 4) {
            s0 += sm.G[b * kGramMax + lane] * sm.vb[b];
            s1 += sm.G[(b + 1) * kGramMax + lane] * sm.vb[b + 1];
            s2 += sm.G[(b + 2) * kGramMax + lane] * sm.vb[b + 2];
            s3 += sm.G[(b + 3) * kGramMax + lane] * sm.vb[b + 3];
        }
        for (; b < k; ++b) s0 += sm.G[b * kGramMax + lane] * sm.vb[b];
        s = (s0 + s1) + (s2 + s3);
    }
    __builtin_amdgcn_wave_barrier();
    return s;
}

// G = X_S^T X_S into sm.G (k <= 16 NB).  Lane l of a wave loads rows
// i0 + 4 (l / 16) .. + 3 of column S[16 bi + l % 16] with one vector load, and
// the 4 MFMAs of a 16-row chunk map their k slot to those rows for both
// operands (both are X_S).  Rows beyond n are zero in X; lanes past the support
// load a valid column and contribute zeros.  The 4 waves split the rows and
// only the lower block triangle is formed.
template <int NB>
__device__ void gram_build_nb(FistaShared &sm, const double *__restrict__ X, int64_t ldx, int64_t np, int k) {
    constexpr int TRI = NB * (NB + 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q = lane >> 4, r = lane & 15;
    f64x4 acc[TRI];
    for (int t = 0; t < TRI; ++t) acc[t] = f64x4{0, 0, 0, 0};
    const double *col[NB];
    bool valid[NB];
    for (int bi = 0; bi < NB; ++bi) {
        const int a = 16 * bi + r;
        valid[bi] = a < k;
        col[bi] = X + (int64_t)sm.idx[valid[bi] ? a : 0] * ldx + 4 * q;
    }
    const int64_t nch = np / 16;
    const int64_t c0 = nch * w / 4, c1 = nch * (w + 1) / 4;
    // two register stages; every load is unconditional (chunk index clamped to
    // the wave's last chunk), so each chunk waits only for its own loads
    double f[2][NB][4];
    auto load = [&](int st, int64_t c) {
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) load4(col[bi] + 16 * c, f[st][bi]);
        __builtin_amdgcn_sched_barrier(0);
    };
    auto compute = [&](int st) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            double x[NB];
#pragma unroll
            for (int bi = 0; bi < NB; ++bi) x[bi] = valid[bi] ? f[st][bi][t] : 0.0;
#pragma unroll
            for (int bi = 0; bi < NB; ++bi)
#pragma unroll
                for (int bj = 0; bj <= bi; ++bj) {
                    const int o = bi * (bi + 1) / 2 + bj;
                    acc[o] = mfma16(x[bi], x[bj], acc[o]);
                }
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    if (c0 < c1) {
        load(0, c0);
        for (int64_t c = c0; c < c1; c += 2) {
            load(1, c + 1 < c1 ? c + 1 : c1 - 1);
            compute(0);
            load(0, c + 2 < c1 ? c + 2 : c1 - 1);
            if (c + 1 < c1) compute(1);
        }
    }
    // cross-wave sum in a fixed order: wave 0 stores, waves 1..3 add in turn
    for (int ww = 0; ww < 4; ++ww) {
        if (w == ww)
            for (int bi = 0; bi < NB; ++bi)
                for (int bj = 0; bj <= bi; ++bj) {
                    const int o = bi * (bi + 1) / 2 + bj;
                    for (int v = 0; v < 4; ++v) {
                        const int row = 16 * bi + acc_row<double>(lane, v), cl = 16 * bj + r;
                        if (row >= k || cl >= k) continue;
                        double x = acc[o][v];
                        double *g1 = &sm.G[cl * kGramMax + row];
                        *g1 = ww == 0 ? x : *g1 + x;
                        if (bi != bj) {
                            double *g2 = &sm.G[row * kGramMax + cl];
                            *g2 = ww == 0 ? x : *g2 + x;
                        }
                    }
                }
        __syncthreads();
    }
}

__device__ void gram_build(FistaShared &sm, const double *__restrict__ X, int64_t ldx, int64_t np, int k) {
    switch ((k + 15) / 16) {
        case 1: gram_build_nb<1>(sm, X, ldx, np, k); break;
        case 2: gram_build_nb<2>(sm, X, ldx, np, k); break;
        case 3: gram_build_nb<3>(sm, X, ldx, np, k); break;
        default: gram_build_nb<4>(sm, X, ldx, np, k); break;
    }
}

// The streaming refinement of one support of k coordinates (k > kGramMax):
// X_S is streamed once per evaluation with all four waves; per-coordinate
// arrays (cur, prev, ext, nxt, grad: k entries each, the support's indices in
// idx) live in LDS for k <= kSMax and in global scratch beyond.  Starts at
// the node iterate brow on S clipped to the box; returns the iterations done,
// the result in cur.
__device__ int fista_stream(const double *__restrict__ X, const double *__restrict__ y,
                            const double *__restrict__ colnrm, const double *__restrict__ brow, const int *idx,
                            int k, double *cur, double *prev, double *ext, double *nxt, double *grad,
                            double *__restrict__ res, double *sh, const FistaArgs &fa) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double fro = 0.0;
    for (int a = tid; a < k; a += 256) {
        double b0 = brow[idx[a]];
        b0 = b0 > fa.M ? fa.M : (b0 < -fa.M ? -fa.M : b0);
        cur[a] = b0;
        prev[a] = b0;
        double cn = colnrm[idx[a]];
        fro += cn * cn;
    }
    fro = bsum(fro, sh);
    double alpha = 4.0 / (fro + 2.0 * fa.l2);
    double Ucur = U_S(X, fa.ldx, y, idx, k, cur, res, false, sh, fa);
    int it = 0;
    while (it < fa.max_iter) {
        double mom = (double)it / ((double)it + 3.0);
        for (int a = tid; a < k; a += 256) ext[a] = cur[a] + mom * (cur[a] - prev[a]);
        __syncthreads();
        double Uext = U_S(X, fa.ldx, y, idx, k, ext, res, true, sh, fa);
        __syncthreads();
        for (int a = w; a < k; a += 4) {
            const double *col = X + (int64_t)idx[a] * fa.ldx;
            double s = 0.0;
            for (int64_t i = lane; i < fa.n; i += 64) s += col[i] * res[i];
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if (lane == 0) grad[a] = s + 2.0 * fa.l2 * ext[a];
        }
        __syncthreads();
        double Unxt = 0.0;
        for (int bt = 0; bt <= 60; ++bt) {
            double gd = 0.0, dd = 0.0;
            for (int a = tid; a < k; a += 256) {
                double v = ext[a] - alpha * grad[a];
                v = v > fa.M ? fa.M : (v < -fa.M ? -fa.M : v);
                nxt[a] = v;
                double d = v - ext[a];
                gd += grad[a] * d;
                dd += d * d;
            }
            gd = bsum(gd, sh);
            dd = bsum(dd, sh);
            Unxt = U_S(X, fa.ldx, y, idx, k, nxt, res, false, sh, fa);
            if (Unxt <= Uext + gd + dd / (2.0 * alpha) || bt == 60) break;
            alpha *= 0.5;
        }
        ++it;
        double dm = 0.0;
        for (int a = tid; a < k; a += 256) dm = fmax(dm, fabs(nxt[a] - cur[a]));
        dm = bmax(dm, sh);
        double dU = fabs(Unxt - Ucur);
        for (int a = tid; a < k; a += 256) {
            prev[a] = cur[a];
            cur[a] = nxt[a];
        }
        __syncthreads();
        Ucur = Unxt;
        if (dU <= fa.tol * (Ucur > 1.0 ? Ucur : 1.0) || dm <= 1e-10) break;
    }
    return it;
}

__global__ __launch_bounds__(256) void k_fista(const double *__restrict__ X, const double *__restrict__ y,
                                               const double *__restrict__ colnrm, const double *__restrict__ c,
                                               double yy, const uint8_t *__restrict__ sup, int64_t lds,
                                               double *__restrict__ beta, int64_t ldb, double *__restrict__ resbuf,
                                               double *__restrict__ obj, int32_t *__restrict__ iters,
                                               int *__restrict__ wlist, int *__restrict__ wcount, FistaArgs fa) {
    __shared__ FistaShared sm;
    const int64_t node = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double *res = resbuf + node * fa.np;
    // compact the support in index order
    int k = 0;
    for (int64_t base = 0; base < fa.p; base += 256) {
        int64_t j = base + tid;
        int f = (j < fa.p) ? sup[node * lds + j] != 0 : 0;
        unsigned long long bal = __ballot(f);
        int before = __popcll(bal & ((1ull << lane) - 1ull));
        __syncthreads();
        if (lane == 0) sm.shw[w] = __popcll(bal);
        __syncthreads();
        int off = k;
        for (int ww = 0; ww < w; ++ww) off += sm.shw[ww];
        if (f && off + before < kSMax) sm.idx[off + before] = (int)j;
        k += sm.shw[0] + sm.shw[1] + sm.shw[2] + sm.shw[3];
    }
    __syncthreads();
    const int *idx = sm.idx;
    if (k > kSMax) {
        // left to k_fista_wide when a wide list is given, else marked unrefined
        if (tid == 0) {
            obj[node] = NAN;
            if (iters) iters[node] = -1;
            if (wlist) wlist[atomicAdd(wcount, 1)] = (int)node;
        }
        return;
    }
    if (k == 0) {
        double s = 0.0;
        for (int64_t i = tid; i < fa.n; i += 256) s += y[i] * y[i];
        s = bsum(s, sm.sh);
        for (int64_t j = tid; j < fa.p; j += 256) beta[node * ldb + j] = 0.0;
        if (tid == 0) {
            obj[node] = 0.5 * s;
            if (iters) iters[node] = 0;
        }
        return;
    }
    if (k <= kGramMax) {
        gram_build(sm, X, fa.ldx, fa.np, k);
        if (w == 0) {
            const bool on = lane < k;
            const double g = on ? c[idx[lane]] : 0.0;
            double cur = 0.0, cn = 0.0;
            if (on) {
                cur = beta[node * ldb + idx[lane]];
                cur = cur > fa.M ? fa.M : (cur < -fa.M ? -fa.M : cur);
                cn = colnrm[idx[lane]];
            }
            double prev = cur;
            double alpha = 4.0 / (wsum(cn * cn) + 2.0 * fa.l2);
            // lane share of U(v) - yy/2 given (G v)_lane
            auto upart = [&](double v, double Gv) { return on ? 0.5 * v * Gv - g * v + fa.l2 * v * v : 0.0; };
            // G cur and G prev are kept, so G ext = G cur + mom (G cur - G prev)
            // needs no product (linearity); each trial forms G nxt
            double Gcur = gram_mv(sm, cur, k, lane), Gprev = Gcur;
            double Ucur = 0.5 * yy + wsum(upart(cur, Gcur));
            int it = 0;
            while (it < fa.max_iter) {
                const double mom = (double)it / ((double)it + 3.0);
                const double ext = cur + mom * (cur - prev);
                const double Gve = Gcur + mom * (Gcur - Gprev);
                const double grad = on ? Gve - g + 2.0 * fa.l2 * ext : 0.0;
                const double Uext = 0.5 * yy + wsum(upart(ext, Gve));
                double Unxt = 0.0, nxt = 0.0, Gn = 0.0, dm = 0.0;
                for (int bt = 0; bt <= 60; ++bt) {
                    double v = ext - alpha * grad;
                    nxt = on ? (v > fa.M ? fa.M : (v < -fa.M ? -fa.M : v)) : 0.0;
                    const double d = nxt - ext;
                    Gn = gram_mv(sm, nxt, k, lane);
                    // independent wave reductions: <grad, d>, |d|^2, U(nxt), max |nxt - cur|
                    const double gd = wsum(grad * d), dd = wsum(d * d);
                    Unxt = 0.5 * yy + wsum(upart(nxt, Gn));
                    dm = wmax(fabs(nxt - cur));
                    if (Unxt <= Uext + gd + dd / (2.0 * alpha) || bt == 60) break;
                    alpha *= 0.5;
                }
                ++it;
                const double dU = fabs(Unxt - Ucur);
                prev = cur;
                cur = nxt;
                Gprev = Gcur;
                Gcur = Gn;
                Ucur = Unxt;
                if (dU <= fa.tol * (Ucur > 1.0 ? Ucur : 1.0) || dm <= 1e-10) break;
            }
            if (on) sm.cur[lane] = cur;
            if (lane == 0) sm.it = it;
        }
        __syncthreads();
    } else {
        const int it = fista_stream(X, y, colnrm, beta + node * ldb, idx, k, sm.cur, sm.prev, sm.ext, sm.nxt, sm.grad,
                                    res, sm.sh, fa);
        if (tid == 0) sm.it = it;
        __syncthreads();
    }
    double f = U_S(X, fa.ldx, y, idx, k, sm.cur, res, false, sm.sh, fa) + fa.l0 * (double)k;
    for (int64_t j = tid; j < fa.p; j += 256) beta[node * ldb + j] = 0.0;
    __syncthreads();
    for (int a = tid; a < k; a += 256) beta[node * ldb + idx[a]] = sm.cur[a];
    if (tid == 0) {
        obj[node] = f;
        if (iters) iters[node] = sm.it;
    }
}

// Supports wider than kSMax: the nodes k_fista listed, one workgroup per node
// in grid-stride order over the list, the support's indices and the five
// per-coordinate arrays in a global slot of stride doubles per workgroup
// (indices first, as ints).  Same iteration as k_fista's streaming form.
__global__ __launch_bounds__(256) void k_fista_wide(const double *__restrict__ X, const double *__restrict__ y,
                                                    const double *__restrict__ colnrm, const uint8_t *__restrict__ sup,
                                                    int64_t lds, double *__restrict__ beta, int64_t ldb,
                                                    double *__restrict__ resbuf, double *__restrict__ obj,
                                                    int32_t *__restrict__ iters, const int *__restrict__ wlist,
                                                    const int *__restrict__ wcount, double *__restrict__ wscr,
                                                    int64_t stride, FistaArgs fa) {
    __shared__ double sh[4];
    __shared__ int shw[4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double *slot = wscr + (int64_t)blockIdx.x * stride;
    int *idx = reinterpret_cast<int *>(slot);
    const int64_t pi = (fa.p + 1) / 2;   // doubles taken by the indices
    double *cur = slot + pi, *prev = cur + fa.p, *ext = prev + fa.p, *nxt = ext + fa.p, *grad = nxt + fa.p;
    const int count = *wcount;
    for (int e = blockIdx.x; e < count; e += gridDim.x) {
        const int64_t node = wlist[e];
        double *res = resbuf + node * fa.np;
        int k = 0;
        for (int64_t base = 0; base < fa.p; base += 256) {
            const int64_t j = base + tid;
            const int f = (j < fa.p) ? sup[node * lds + j] != 0 : 0;
            const unsigned long long bal = __ballot(f);
            const int before = __popcll(bal & ((1ull << lane) - 1ull));
            __syncthreads();
            if (lane == 0) shw[w] = __popcll(bal);
            __syncthreads();
            int off = k;
            for (int ww = 0; ww < w; ++ww) off += shw[ww];
            if (f) idx[off + before] = (int)j;
            k += shw[0] + shw[1] + shw[2] + shw[3];
        }
        __syncthreads();
        const int it = fista_stream(X, y, colnrm, beta + node * ldb, idx, k, cur, prev, ext, nxt, grad, res, sh, fa);
        const double f = U_S(X, fa.ldx, y, idx, k, cur, res, false, sh, fa) + fa.l0 * (double)k;
        for (int64_t j = tid; j < fa.p; j += 256) beta[node * ldb + j] = 0.0;
        __syncthreads();
        for (int a = tid; a < k; a += 256) beta[node * ldb + idx[a]] = cur[a];
        if (tid == 0) {
            obj[node] = f;
            if (iters) iters[node] = it;
        }
        __syncthreads();
    }
}

__global__ void k_zero_int(int *v) { *v = 0; }

template <class T>
__global__ void k_state_f64(const T *__restrict__ src, int64_t lds, double *__restrict__ dst, int64_t ldd, int64_t K,
                            int64_t p) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < K * p; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t k = idx / p, j = idx % p;
        dst[k * ldd + j] = (double)src[k * lds + j];
    }
}

// Exact box-constrained ridge on one support, single workgroup:
// H = X_S^T X_S + 2 l2 I, g = X_S^T y; Cholesky solve; if the box binds,
// coordinate descent on 1/2 b^T H b - g^T b over [-M, M]^k.
__global__ __launch_bounds__(256) void k_exact(const double *__restrict__ X, int64_t ldx, const double *__restrict__ y,
                                               const double *__restrict__ c, const int *__restrict__ idx, int k,
                                               double *__restrict__ H, double *__restrict__ L,
                                               double *__restrict__ bsol, double *__restrict__ res,
                                               double *__restrict__ out, FistaArgs fa) {
    __shared__ double sh[4];
    __shared__ int flag;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int e = w; e < k * k; e += 4) {
        int a = e % k, b = e / k;
        if (b > a) continue;
        const double *ca = X + (int64_t)idx[a] * ldx, *cb = X + (int64_t)idx[b] * ldx;
        double s = 0.0;
        for (int64_t i = lane; i < fa.n; i += 64) s += ca[i] * cb[i];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) {
            double v = s + (a == b ? 2.0 * fa.l2 : 0.0);
            H[a + b * k] = v;
            H[b + a * k] = v;
        }
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += 256) L[e] = H[e];
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (tid == 0) {
            double d = L[j + j * k];
            if (!(d > 0.0)) { flag = 1; d = 1.0; }
            L[j + j * k] = sqrt(d);
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < k; i += 256) L[i + j * k] /= L[j + j * k];
        __syncthreads();
        int rem = k - j - 1;
        for (int e = tid; e < rem * rem; e += 256) {
            int i = j + 1 + e % rem, m = j + 1 + e / rem;
            if (m <= i) L[i + m * k] -= L[i + j * k] * L[m + j * k];
        }
        __syncthreads();
    }
    if (tid == 0) {
        for (int a = 0; a < k; ++a) bsol[a] = c[idx[a]];
        if (!flag) {
            for (int i = 0; i < k; ++i) {
                double s = bsol[i];
                for (int m = 0; m < i; ++m) s -= L[i + m * k] * bsol[m];
                bsol[i] = s / L[i + i * k];
            }
            for (int i = k - 1; i >= 0; --i) {
                double s = bsol[i];
                for (int m = i + 1; m < k; ++m) s -= L[m + i * k] * bsol[m];
                bsol[i] = s / L[i + i * k];
            }
        }
        int boxed = flag;
        for (int a = 0; a < k; ++a) if (fabs(bsol[a]) > fa.M) boxed = 1;
        if (flag) for (int a = 0; a < k; ++a) bsol[a] = 0.0;
        flag = boxed;
    }
    __syncthreads();
    if (flag) {
        for (int a = tid; a < k; a += 256) bsol[a] = fmin(fa.M, fmax(-fa.M, bsol[a]));
        __syncthreads();
        for (int sweep = 0; sweep < 200000; ++sweep) {
            double dmax = 0.0, bm = 0.0;
            for (int a = 0; a < k; ++a) {
                double part = 0.0;
                for (int b = tid; b < k; b += 256) if (b != a) part += H[b * k + a] * bsol[b];
                part = bsum(part, sh);
                double nv = (c[idx[a]] - part) / H[a * k + a];
                nv = fmin(fa.M, fmax(-fa.M, nv));
                dmax = fmax(dmax, fabs(nv - bsol[a]));
                bm = fmax(bm, fabs(nv));
                __syncthreads();
                if (tid == 0) bsol[a] = nv;
                __syncthreads();
            }
            if (dmax <= 1e-16 * (bm > 1.0 ? bm : 1.0)) break;
        }
    }
    __syncthreads();
    double rr = 0.0;
    for (int64_t i = tid; i < fa.n; i += 256) {
        double s = 0.0;
        for (int a = 0; a < k; ++a) s += X[(int64_t)idx[a] * ldx + i] * bsol[a];
        double r = s - y[i];
        rr += r * r;
    }
    double bb = 0.0;
    for (int a = tid; a < k; a += 256) bb += bsol[a] * bsol[a];
    rr = bsum(rr, sh);
    bb = bsum(bb, sh);
    if (tid == 0) *out = 0.5 * rr + fa.l2 * bb + fa.l0 * (double)k;
    (void)res;
}

}  // namespace

void run_round_branch(l0l2_ctx *ctx, int K, const uint8_t *codes, int64_t ld_codes, const void *beta,
                      int64_t ld_beta, uint8_t *support, int32_t *support_size, int32_t *branch_j, int32_t *z_up, int32_t *nfree) {
    Instance &in = ctx->inst;
    RoundArgs ra{in.mp.s, in.mp.M, in.mp.free_quad, in.p};
    if (K <= 0) return;
    prof_begin(ctx, PROF_ROUND);
    if (in.prec == L0L2_FP64)
        hipLaunchKernelGGL(k_round_branch<double>, dim3((unsigned)K), dim3(256), 0, ctx->stream, codes, ld_codes,
                           (const double *)beta, ld_beta, support, support_size, branch_j, z_up, nfree, ra);
    else
        hipLaunchKernelGGL(k_round_branch<float>, dim3((unsigned)K), dim3(256), 0, ctx->stream, codes, ld_codes,
                           (const float *)beta, ld_beta, support, support_size, branch_j, z_up, nfree, ra);
    prof_end(ctx, PROF_ROUND);
    HIPCHK(hipGetLastError());
}

void run_fista(l0l2_ctx *ctx, int K, const uint8_t *support, int64_t ld_support, double *beta, int64_t ld_beta,
               const l0l2_fista_opts &o, double *obj, int32_t *iters, double *resbuf) {
    Instance &in = ctx->inst;
    if (K <= 0) return;
    // resbuf: K rows of np doubles supplied by the caller (the allocation-free
    // entry point), else the workspace's, grown here
    const bool own = resbuf == nullptr;
    if (own) {
        ctx->ws.fista.ensure(sizeof(double) * (size_t)K * in.np);
        resbuf = ctx->ws.fista.as<double>();
    }
    FistaArgs fa{in.mp.l0, in.mp.l2, in.mp.M, o.tol, o.max_iter, in.n, in.np, in.p, in.ldx};
    // supports wider than kSMax (possible only when p > kSMax) go to the wide
    // kernel, whose slots (at most 64, at most 256 MiB) the workspace holds;
    // the allocation-free form leaves them unrefined
    const bool wide = own && in.p > kSMax;
    int *wlist = nullptr, *wcount = nullptr;
    int slots = 0;
    const int64_t stride = 5 * in.p + (in.p + 1) / 2;
    if (wide) {
        slots = (int)std::min<int64_t>({(int64_t)K, 64, std::max<int64_t>(1, (256ll << 20) / (8 * stride))});
        ctx->ws.fista_wide.ensure(sizeof(double) * (size_t)slots * stride);
        ctx->ws.fista_list.ensure(sizeof(int) * ((size_t)K + 1));
        wcount = ctx->ws.fista_list.as<int>();
        wlist = wcount + 1;
    }
    if (own) prof_begin(ctx, PROF_FISTA);
    if (wide) hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, ctx->stream, wcount);
    hipLaunchKernelGGL(k_fista, dim3((unsigned)K), dim3(256), 0, ctx->stream, in.X64.as<double>(), in.y64.as<double>(),
                       in.colnrm.as<double>(), in.c64.as<double>(), in.yy, support, ld_support, beta, ld_beta,
                       resbuf, obj, iters, wlist, wcount, fa);
    if (wide)
        hipLaunchKernelGGL(k_fista_wide, dim3((unsigned)slots), dim3(256), 0, ctx->stream, in.X64.as<double>(),
                           in.y64.as<double>(), in.colnrm.as<double>(), support, ld_support, beta, ld_beta, resbuf, obj,
                           iters, (const int *)wlist, (const int *)wcount, ctx->ws.fista_wide.as<double>(), stride, fa);
    if (own) prof_end(ctx, PROF_FISTA);
    HIPCHK(hipGetLastError());
}

double run_exact_objective(l0l2_ctx *ctx, const uint8_t *support_host, double *beta_host) {
    Instance &in = ctx->inst;
    hipStream_t s = ctx->stream;
    std::vector<int> idx;
    for (int64_t j = 0; j < in.p; ++j)
        if (support_host[j]) idx.push_back((int)j);
    const int k = (int)idx.size();
    for (int64_t j = 0; j < in.p; ++j) beta_host[j] = 0.0;
    DevBuf didx, H, L, b, out;
    didx.ensure(sizeof(int) * (size_t)std::max(k, 1));
    H.ensure(sizeof(double) * (size_t)std::max(k * k, 1));
    L.ensure(sizeof(double) * (size_t)std::max(k * k, 1));
    b.ensure(sizeof(double) * (size_t)std::max(k, 1));
    out.ensure(sizeof(double));
    if (k) HIPCHK(hipMemcpyAsync(didx.ptr, idx.data(), sizeof(int) * k, hipMemcpyHostToDevice, s));
    FistaArgs fa{in.mp.l0, in.mp.l2, in.mp.M, 0.0, 0, in.n, in.np, in.p, in.ldx};
    hipLaunchKernelGGL(k_exact, dim3(1), dim3(256), 0, s, in.X64.as<double>(), in.ldx, in.y64.as<double>(),
                       in.c64.as<double>(), didx.as<int>(), k, H.as<double>(), L.as<double>(), b.as<double>(),
                       (double *)nullptr, out.as<double>(), fa);
    HIPCHK(hipGetLastError());
    double f = 0.0;
    std::vector<double> hb((size_t)std::max(k, 1));
    HIPCHK(hipMemcpyAsync(&f, out.ptr, sizeof(double), hipMemcpyDeviceToHost, s));
    if (k) HIPCHK(hipMemcpyAsync(hb.data(), b.ptr, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int a = 0; a < k; ++a) beta_host[idx[a]] = hb[a];
    return f;
}

void state_to_f64(l0l2_ctx *ctx, int K, const void *src, int64_t ld_src, double *dst, int64_t ld_dst) {
    Instance &in = ctx->inst;
    unsigned g = (unsigned)std::min<int64_t>(((int64_t)K * in.p + 255) / 256, 65536);
    if (K <= 0) return;
    if (in.prec == L0L2_FP64)
        hipLaunchKernelGGL(k_state_f64<double>, dim3(g), dim3(256), 0, ctx->stream, (const double *)src, ld_src, dst,
                           ld_dst, (int64_t)K, in.p);
    else
        hipLaunchKernelGGL(k_state_f64<float>, dim3(g), dim3(256), 0, ctx->stream, (const float *)src, ld_src, dst,
                           ld_dst, (int64_t)K, in.p);
    HIPCHK(hipGetLastError());
}

}  // namespace l0l2
