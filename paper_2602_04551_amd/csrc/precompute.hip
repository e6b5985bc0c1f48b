// Once-per-instance precompute (Sec. 3.1.1, update for b): c = X^T y, column
// norms, S = X X^T + rho I, its Cholesky factor L, and the folded operand
// Xh = L^{-1} X so that D w = (w - Xh^T (Xh w)) / rho for D = (X^T X + rho I)^{-1}
// (the Woodbury identity with the 1/rho factor; Xh^T Xh = X^T S^{-1} X).
#include <algorithm>
#include <cmath>
#include <vector>
#include <cstring>

#include "device_math.hpp"
#include "internal.hpp"

namespace l0l2 {

namespace {

// dst (np x pp, column stride ld) <- src (n x p, ld = n), zero padding.
__global__ void k_pad_copy(const double *__restrict__ src, int64_t n, int64_t p, double *__restrict__ dst,
                           int64_t np, int64_t pp, int64_t ld) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = np * pp;
    for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx % np, j = idx / np;
        dst[i + j * ld] = (i < n && j < p) ? src[i + j * n] : 0.0;
    }
}

// One wave per column: c_j = X_j^T y and ||X_j||.
__global__ __launch_bounds__(256) void k_colstats(const double *__restrict__ X, int64_t ldx,
                                                  const double *__restrict__ y, int64_t np, int64_t pp,
                                                  double *__restrict__ c, double *__restrict__ nrm) {
    int lane = threadIdx.x & 63;
    int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= pp) return;
    const double *col = X + j * ldx;
    double s = 0.0, q = 0.0;
    for (int64_t i = lane; i < np; i += 64) {
        double x = col[i];
        s += x * y[i];
        q += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off);
        q += __shfl_xor(q, off);
    }
    if (lane == 0) {
        c[j] = s;
        nrm[j] = sqrt(q);
    }
}

// C[i + j*ldc] = alpha * sum_k A(i,k) B(k,j) + beta * C[i + j*ldc] for i < M, j < N,
// A(i,k) = A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj].  64x64 tiles, FP64 MFMA.
__global__ __launch_bounds__(256) void k_dgemm(int64_t M, int64_t N, int64_t K, double alpha,
                                               const double *__restrict__ A, int64_t sai, int64_t sak,
                                               const double *__restrict__ B, int64_t sbk, int64_t sbj,
                                               double beta, double *__restrict__ C, int64_t ldc) {
    __shared__ double As[16][64 + 1];
    __shared__ double Bs[16][64 + 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int64_t m0 = (int64_t)blockIdx.x * 64, n0 = (int64_t)blockIdx.y * 64;
    f64x4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0, 0, 0, 0};
    const bool a_i_fast = (sai == 1);
    const bool b_j_fast = (sbj == 1);
    for (int64_t k0 = 0; k0 < K; k0 += 16) {
        for (int r = 0; r < 4; ++r) {
            int e = tid + 256 * r;
            int il, kl;
            if (a_i_fast) { il = e & 63; kl = e >> 6; } else { kl = e & 15; il = e >> 4; }
            int64_t gi = m0 + il, gk = k0 + kl;
            As[kl][il] = (gi < M && gk < K) ? A[gi * sai + gk * sak] : 0.0;
            int jl, kl2;
            if (b_j_fast) { jl = e & 63; kl2 = e >> 6; } else { kl2 = e & 15; jl = e >> 4; }
            int64_t gj = n0 + jl, gk2 = k0 + kl2;
            Bs[kl2][jl] = (gj < N && gk2 < K) ? B[gk2 * sbk + gj * sbj] : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < 4; ++kk) {
            int krow = kk * 4 + (lane >> 4);
            double av[2], bv[2];
            for (int a = 0; a < 2; ++a) av[a] = As[krow][wm * 32 + a * 16 + (lane & 15)];
            for (int b = 0; b < 2; ++b) bv[b] = Bs[krow][wn * 32 + b * 16 + (lane & 15)];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int v = 0; v < 4; ++v) {
                int64_t gi = m0 + wm * 32 + a * 16 + acc_row<double>(lane, v);
                int64_t gj = n0 + wn * 32 + b * 16 + (lane & 15);
                if (gi < M && gj < N) {
                    double old = beta != 0.0 ? C[gi + gj * ldc] : 0.0;
                    C[gi + gj * ldc] = alpha * acc[a][b][v] + beta * old;
                }
            }
}

// In-place lower Cholesky of the nb x nb diagonal block at S + kb*(ld+1).
__global__ __launch_bounds__(256) void k_potrf_diag(double *S, int64_t ld, int64_t kb, int nb, int *fail_flag) {
    __shared__ double L[64][65];
    const int tid = threadIdx.x;
    double *blk = S + kb * ld + kb;
    for (int e = tid; e < nb * nb; e += 256) {
        int i = e % nb, j = e / nb;
        L[i][j] = blk[i + j * ld];
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (tid == 0) {
            double d = L[j][j];
            if (!(d > 0.0)) {
                *fail_flag = 1;
                d = 1.0;
            }
            L[j][j] = sqrt(d);
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < nb; i += 256) L[i][j] /= L[j][j];
        __syncthreads();
        int rem = nb - j - 1;
        for (int e = tid; e < rem * rem; e += 256) {
            int i = j + 1 + e % rem, k = j + 1 + e / rem;
            if (k <= i) L[i][k] -= L[i][j] * L[k][j];
        }
        __syncthreads();
    }
    for (int e = tid; e < nb * nb; e += 256) {
        int i = e % nb, j = e / nb;
        blk[i + j * ld] = (i >= j) ? L[i][j] : 0.0;
    }
}

// Rows [r0, r0 + nrows) of the panel S[:, kb:kb+nb] <- panel * L_kk^{-T}: one
// thread per row, row data in LDS.
__global__ __launch_bounds__(64) void k_trsm_panel(double *S, int64_t ld, int64_t kb, int nb, int64_t r0,
                                                   int64_t nrows) {
    __shared__ double L[64][65];
    __shared__ double Xr[64][65];
    const int t = threadIdx.x;
    const double *Lkk = S + kb * ld + kb;
    for (int e = t; e < nb * nb; e += 64) {
        int i = e % nb, j = e / nb;
        L[i][j] = Lkk[i + j * ld];
    }
    int64_t row = r0 + (int64_t)blockIdx.x * 64 + t;
    bool ok = (row - r0) < nrows;
    for (int j = 0; j < nb; ++j) Xr[t][j] = ok ? S[row + (kb + j) * ld] : 0.0;
    __syncthreads();
    if (!ok) return;
    for (int j = 0; j < nb; ++j) {
        double s = Xr[t][j];
        for (int k = 0; k < j; ++k) s -= Xr[t][k] * L[j][k];
        Xr[t][j] = s / L[j][j];
    }
    for (int j = 0; j < nb; ++j) S[row + (kb + j) * ld] = Xr[t][j];
}

// Columns of the row block X[kb:kb+nb, :] <- L_kk^{-1} X[kb:kb+nb, :] (forward
// substitution, one thread per column).
__global__ __launch_bounds__(64) void k_trsv_rows(const double *S, int64_t lds, double *X, int64_t ldx,
                                                  int64_t kb, int nb, int64_t ncols) {
    __shared__ double L[64][65];
    __shared__ double Xc[64][65];
    const int t = threadIdx.x;
    const double *Lkk = S + kb * lds + kb;
    for (int e = t; e < nb * nb; e += 64) {
        int i = e % nb, j = e / nb;
        L[i][j] = Lkk[i + j * lds];
    }
    int64_t col = (int64_t)blockIdx.x * 64 + t;
    bool ok = col < ncols;
    for (int i = 0; i < nb; ++i) Xc[t][i] = ok ? X[kb + i + col * ldx] : 0.0;
    __syncthreads();
    if (!ok) return;
    for (int i = 0; i < nb; ++i) {
        double s = Xc[t][i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * Xc[t][k];
        Xc[t][i] = s / L[i][i];
    }
    for (int i = 0; i < nb; ++i) X[kb + i + col * ldx] = Xc[t][i];
}

// dst (row-major, rows of stride ldd) <- src (np x pp column-major, column
// stride lds), by 32 x 32 tiles through LDS so both sides are coalesced.
template <class TS, class TD>
__global__ __launch_bounds__(256) void k_transpose(const TS *__restrict__ src, int64_t lds, TD *__restrict__ dst,
                                                   int64_t ldd) {
    __shared__ TD t[32][33];
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) t[r][tx] = (TD)src[(j0 + r) * lds + i0 + tx];
    __syncthreads();
    for (int r = ty; r < 32; r += 8) dst[(i0 + r) * ldd + j0 + tx] = t[tx][r];
}

template <class TS, class TD>
void transpose(hipStream_t st, const TS *src, int64_t lds, TD *dst, int64_t ldd, int64_t np, int64_t pp) {
    hipLaunchKernelGGL((k_transpose<TS, TD>), dim3((unsigned)(np / 32), (unsigned)(pp / 32)), dim3(256), 0, st, src,
                       lds, dst, ldd);
    HIPCHK(hipGetLastError());
}

__global__ void k_add_diag(double *S, int64_t ld, int64_t n, double r) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) S[i + i * ld] += r;
}

__global__ void k_to_f32(const double *__restrict__ src, float *__restrict__ dst, int64_t total) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) dst[idx] = (float)src[idx];
}

// FP32 rounding of the np x pp column-major src (column stride lds) into dst
// (column stride ldd).
__global__ void k_to_f32_cols(const double *__restrict__ src, int64_t lds, float *__restrict__ dst, int64_t ldd,
                              int64_t np, int64_t pp) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < np * pp; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx % np, j = idx / np;
        dst[i + j * ldd] = (float)src[i + j * lds];
    }
}

// Two-term BF16 split x = hi + lo of the np x pp column-major src (column
// stride lds), stored column-major (stride ldc) and row-major (stride ldr).
__global__ void k_to_bf16x2(const double *__restrict__ src, int64_t lds, __bf16 *__restrict__ col_hi,
                            __bf16 *__restrict__ col_lo, int64_t ldc, __bf16 *__restrict__ row_hi,
                            __bf16 *__restrict__ row_lo, int64_t ldr, int64_t np, int64_t pp) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = np * pp;
    for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx % np, j = idx / np;
        double x = src[i + j * lds];
        __bf16 hi = (__bf16)(float)x;
        __bf16 lo = (__bf16)(float)(x - (double)(float)hi);
        col_hi[i + j * ldc] = hi;
        col_lo[i + j * ldc] = lo;
        row_hi[i * ldr + j] = hi;
        row_lo[i * ldr + j] = lo;
    }
}

// FP8 e4m3 (OCP): largest finite magnitude.
constexpr double kFp8Max = 448.0;

// One wave per column: s_j = max_i |Xh_ij| / 448 (1 for an all-zero column).
__global__ __launch_bounds__(256) void k_fp8_scales(const double *__restrict__ X, int64_t ldx, int64_t np,
                                                    int64_t pp, float *__restrict__ s) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= pp) return;
    double mx = 0.0;
    for (int64_t i = lane; i < np; i += 64) mx = fmax(mx, fabs(X[i + j * ldx]));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if (lane == 0) s[j] = mx > 0.0 ? (float)(mx / kFp8Max) : 1.0f;
}

// q_ij = e4m3(Xh_ij / s_j) (round to nearest even; the quotient is clamped to
// the finite range, the conversion gives NaN beyond it), stored column-major
// (stride ldc bytes) and row-major (stride ldr bytes).
__global__ void k_to_fp8(const double *__restrict__ X, int64_t ldx, const float *__restrict__ s,
                         uint8_t *__restrict__ col, int64_t ldc, uint8_t *__restrict__ row, int64_t ldr, int64_t np,
                         int64_t pp) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; idx < np * pp; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % np, j = idx / np;
        const double t = X[i + j * ldx] / (double)s[j];
        const float v = (float)fmin(kFp8Max, fmax(-kFp8Max, t));
        const uint8_t q = (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, v, 0, false) & 0xFF);
        col[i + j * ldc] = q;
        row[i * ldr + j] = q;
    }
}

void dgemm(hipStream_t st, int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t sai,
           int64_t sak, const double *B, int64_t sbk, int64_t sbj, double beta, double *C, int64_t ldc) {
    if (M <= 0 || N <= 0) return;
    dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64));
    hipLaunchKernelGGL(k_dgemm, grid, dim3(256), 0, st, M, N, K, alpha, A, sai, sak, B, sbk, sbj, beta, C, ldc);
    HIPCHK(hipGetLastError());
}

}  // namespace

MethodParams make_params(double l0, double l2, double M, double rho) {
    MethodParams q{};
    q.l0 = l0; q.l2 = l2; q.M = M; q.rho = rho;
    q.s = sqrt(l0 / l2);
    q.free_quad = q.s <= M;
    q.a = 2.0 * sqrt(l0 * l2) / rho;
    q.a_plus_s = q.a + q.s;
    q.ridge = rho / (rho + 2.0 * l2);
    q.thr_lin = l0 / (M * rho) + l2 * M / rho;
    q.thr_free = q.free_quad ? q.a : q.thr_lin;
    q.thr_free_M = q.thr_free + M;
    q.two_M_l2 = 2.0 * M * l2;
    q.four_l2 = 4.0 * l2;
    q.l2_M2 = l2 * M * M;
    q.psi_lin = q.free_quad ? 2.0 * sqrt(l0 * l2) : (l0 / M + l2 * M);
    return q;
}

void set_penalties(l0l2_ctx *ctx, double l0, double l2, double M) {
    Instance &in = ctx->inst;
    // the captured blocks of sweeps hold the old scalars as kernel arguments
    HIPCHK(hipStreamSynchronize(ctx->stream));
    drop_graphs(ctx);
    in.mp = make_params(l0, l2, M, in.mp.rho);
}

double lambda0_max(l0l2_ctx *ctx) {
    Instance &in = ctx->inst;
    const int64_t p = in.p;
    std::vector<double> c((size_t)p), nrm((size_t)p);
    HIPCHK(hipMemcpyAsync(c.data(), in.c64.ptr, sizeof(double) * p, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(nrm.data(), in.colnrm.ptr, sizeof(double) * p, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    double best = 0.0;
    for (int64_t j = 0; j < p; ++j) {
        const double D = nrm[(size_t)j] * nrm[(size_t)j] + 2.0 * in.mp.l2;
        double b = c[(size_t)j] / D;
        b = b > in.mp.M ? in.mp.M : (b < -in.mp.M ? -in.mp.M : b);
        best = std::max(best, b * c[(size_t)j] - 0.5 * D * b * b);
    }
    return best;
}

void set_data(l0l2_ctx *ctx, const double *X, const double *y, int64_t n, int64_t p, double l0, double l2,
              double M, double rho, int prec, int on_device) {
    Instance &in = ctx->inst;
    hipStream_t st = ctx->stream;
    ctx->has_data = false;
    // the per-batch workspace is sized for the previous instance: drop it
    ctx->ws.cap = 0;
    ctx->ws.have_root = false;
    drop_graphs(ctx);
    in.tiles.clear();
    in.tuned_K = 0;
    in.gram_built = false;
    in.form_pick = 0;
    in.form_ms[0] = in.form_ms[1] = 0.0;
    in.n = n;
    in.p = p;
    in.np = round_up(n, kPadRows);
    in.pp = round_up(p, kPadRows);
    in.prec = prec;
    in.mp = make_params(l0, l2, M, rho);
    const int64_t np = in.np, pp = in.pp;
    const int64_t ws_elem = prec == L0L2_FP64 ? 8 : (prec == L0L2_FP32 ? 4 : 2);   // working-precision bytes
    in.ldx = ld_pad(np, 8);
    in.ldxr = ld_pad(pp, 8);
    in.ldw = prec == L0L2_FP64 ? in.ldx : ld_pad(np, ws_elem);
    in.ldwr = prec == L0L2_FP64 ? in.ldxr : ld_pad(pp, ws_elem);
    in.ldp = ld_pad(pp, prec == L0L2_FP64 ? 8 : 4);
    in.ldu = ld_pad(np, prec == L0L2_FP64 ? 8 : 4);
    in.ldu64 = ld_pad(np, 8);
    const int64_t ldx = in.ldx, ldxr = in.ldxr, ldp = in.ldp;

    // Stage X and y on the device unpadded, then pad.
    DevBuf Xraw, yraw;
    const double *dX = X, *dy = y;
    if (!on_device) {
        Xraw.ensure(sizeof(double) * (size_t)(n * p));
        yraw.ensure(sizeof(double) * (size_t)n);
        HIPCHK(hipMemcpyAsync(Xraw.ptr, X, sizeof(double) * (size_t)(n * p), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(yraw.ptr, y, sizeof(double) * (size_t)n, hipMemcpyHostToDevice, st));
        dX = Xraw.as<double>();
        dy = yraw.as<double>();
    }
    // every buffer is cleared first: the gaps between the padded extent and the
    // leading dimension hold zeros
    in.X64.ensure(sizeof(double) * (size_t)(ldx * pp));
    in.y64.ensure(sizeof(double) * (size_t)np);
    in.c64.ensure(sizeof(double) * (size_t)ldp);
    in.colnrm.ensure(sizeof(double) * (size_t)ldp);
    HIPCHK(hipMemsetAsync(in.X64.ptr, 0, sizeof(double) * (size_t)(ldx * pp), st));
    HIPCHK(hipMemsetAsync(in.c64.ptr, 0, sizeof(double) * (size_t)ldp, st));
    HIPCHK(hipMemsetAsync(in.colnrm.ptr, 0, sizeof(double) * (size_t)ldp, st));
    hipLaunchKernelGGL(k_pad_copy, dim3(2048), dim3(256), 0, st, dX, n, p, in.X64.as<double>(), np, pp, ldx);
    hipLaunchKernelGGL(k_pad_copy, dim3(64), dim3(256), 0, st, dy, n, (int64_t)1, in.y64.as<double>(), np,
                       (int64_t)1, np);
    hipLaunchKernelGGL(k_colstats, dim3((unsigned)((pp + 3) / 4)), dim3(256), 0, st, in.X64.as<double>(), ldx,
                       in.y64.as<double>(), np, pp, in.c64.as<double>(), in.colnrm.as<double>());
    HIPCHK(hipGetLastError());

    // S = X X^T + rho I (n x n, ld = np), then its Cholesky factor in place.
    DevBuf S, flag;
    S.ensure(sizeof(double) * (size_t)(np * np));
    flag.ensure(sizeof(int));
    HIPCHK(hipMemsetAsync(S.ptr, 0, sizeof(double) * (size_t)(np * np), st));
    HIPCHK(hipMemsetAsync(flag.ptr, 0, sizeof(int), st));
    const double *X64 = in.X64.as<double>();
    dgemm(st, n, n, p, 1.0, X64, 1, ldx, X64, ldx, 1, 0.0, S.as<double>(), np);
    hipLaunchKernelGGL(k_add_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, S.as<double>(), np, n,
                       rho);
    HIPCHK(hipGetLastError());
    double *Sd = S.as<double>();
    for (int64_t kb = 0; kb < n; kb += 64) {
        int nb = (int)std::min<int64_t>(64, n - kb);
        hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, Sd, np, kb, nb, flag.as<int>());
        int64_t r0 = kb + nb, rem = n - r0;
        if (rem > 0) {
            hipLaunchKernelGGL(k_trsm_panel, dim3((unsigned)((rem + 63) / 64)), dim3(64), 0, st, Sd, np, kb, nb,
                               r0, rem);
            // trailing update S[r0:, r0:] -= P P^T, P = S[r0:, kb:kb+nb]
            const double *P = Sd + r0 + kb * np;
            dgemm(st, rem, rem, nb, -1.0, P, 1, np, P, np, 1, 1.0, Sd + r0 + r0 * np, np);
        }
        HIPCHK(hipGetLastError());
    }
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, flag.ptr, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hflag) fail(L0L2_E_NUMERIC, "Cholesky of X X^T + rho I failed (not positive definite)");

    // Xh = L^{-1} X, blocked forward substitution over row blocks of 64.
    // FP64 mode keeps it as the sweep operand; the reduced-precision modes keep
    // it for the anchored sweeps.  Column stride ldx, as X64.
    double *Xh;
    if (prec == L0L2_FP64) {
        in.Xh.ensure(sizeof(double) * (size_t)(ldx * pp));
        Xh = in.Xh.as<double>();
    } else {
        in.Xh64.ensure(sizeof(double) * (size_t)(ldx * pp));
        Xh = in.Xh64.as<double>();
    }
    HIPCHK(hipMemcpyAsync(Xh, X64, sizeof(double) * (size_t)(ldx * pp), hipMemcpyDeviceToDevice, st));
    for (int64_t kb = 0; kb < n; kb += 64) {
        int nb = (int)std::min<int64_t>(64, n - kb);
        hipLaunchKernelGGL(k_trsv_rows, dim3((unsigned)((p + 63) / 64)), dim3(64), 0, st, Sd, np, Xh, ldx, kb, nb,
                           p);
        int64_t r0 = kb + nb, rem = n - r0;
        if (rem > 0) {
            // X[r0:, :] -= L[r0:, kb:kb+nb] * Xh[kb:kb+nb, :]
            dgemm(st, rem, p, nb, -1.0, Sd + r0 + kb * np, 1, np, Xh + kb, 1, ldx, 1.0, Xh + r0, ldx);
        }
        HIPCHK(hipGetLastError());
    }
    // row-major copies for the contractions over p (gaps past pp cleared)
    in.X64R.ensure(sizeof(double) * (size_t)(np * ldxr));
    HIPCHK(hipMemsetAsync(in.X64R.ptr, 0, sizeof(double) * (size_t)(np * ldxr), st));
    transpose<double, double>(st, X64, ldx, in.X64R.as<double>(), ldxr, np, pp);
    if (prec == L0L2_FP64) {
        in.XhRw.ensure(sizeof(double) * (size_t)(np * ldxr));
        HIPCHK(hipMemsetAsync(in.XhRw.ptr, 0, sizeof(double) * (size_t)(np * ldxr), st));
        transpose<double, double>(st, Xh, ldx, in.XhRw.as<double>(), ldxr, np, pp);
    } else {
        in.Xh64R.ensure(sizeof(double) * (size_t)(np * ldxr));
        HIPCHK(hipMemsetAsync(in.Xh64R.ptr, 0, sizeof(double) * (size_t)(np * ldxr), st));
        transpose<double, double>(st, Xh, ldx, in.Xh64R.as<double>(), ldxr, np, pp);
    }
    const int64_t ldw = in.ldw, ldwr = in.ldwr;
    if (prec == L0L2_FP32) {
        in.XhRw.ensure(sizeof(float) * (size_t)(np * ldwr));
        HIPCHK(hipMemsetAsync(in.XhRw.ptr, 0, sizeof(float) * (size_t)(np * ldwr), st));
        transpose<double, float>(st, Xh, ldx, in.XhRw.as<float>(), ldwr, np, pp);
        in.Xh.ensure(sizeof(float) * (size_t)(ldw * pp));
        HIPCHK(hipMemsetAsync(in.Xh.ptr, 0, sizeof(float) * (size_t)(ldw * pp), st));
        hipLaunchKernelGGL(k_to_f32_cols, dim3(4096), dim3(256), 0, st, Xh, ldx, in.Xh.as<float>(), ldw, np, pp);
        in.cst.ensure(sizeof(float) * (size_t)ldp);
        hipLaunchKernelGGL(k_to_f32, dim3(64), dim3(256), 0, st, in.c64.as<double>(), in.cst.as<float>(), ldp);
    } else if (prec == L0L2_BF16) {
        const size_t nbc = sizeof(__bf16) * (size_t)(ldw * pp), nbr = sizeof(__bf16) * (size_t)(np * ldwr);
        in.Xh.ensure(nbc);
        in.XhLo.ensure(nbc);
        in.XhR.ensure(nbr);
        in.XhRLo.ensure(nbr);
        HIPCHK(hipMemsetAsync(in.Xh.ptr, 0, nbc, st));
        HIPCHK(hipMemsetAsync(in.XhLo.ptr, 0, nbc, st));
        HIPCHK(hipMemsetAsync(in.XhR.ptr, 0, nbr, st));
        HIPCHK(hipMemsetAsync(in.XhRLo.ptr, 0, nbr, st));
        hipLaunchKernelGGL(k_to_bf16x2, dim3(4096), dim3(256), 0, st, Xh, ldx, in.Xh.as<__bf16>(),
                           in.XhLo.as<__bf16>(), ldw, in.XhR.as<__bf16>(), in.XhRLo.as<__bf16>(), ldwr, np, pp);
        in.cst.ensure(sizeof(float) * (size_t)ldp);
        hipLaunchKernelGGL(k_to_f32, dim3(64), dim3(256), 0, st, in.c64.as<double>(), in.cst.as<float>(), ldp);
    } else if (prec == L0L2_FP8) {
        in.ldqr = ld_pad(pp, 1);
        in.ldqc = ld_pad(np, 1);
        in.qs.ensure(sizeof(float) * (size_t)ldp);
        in.qR.ensure((size_t)(np * in.ldqr));
        in.qC.ensure((size_t)(in.ldqc * pp));
        HIPCHK(hipMemsetAsync(in.qs.ptr, 0, sizeof(float) * (size_t)ldp, st));
        HIPCHK(hipMemsetAsync(in.qR.ptr, 0, (size_t)(np * in.ldqr), st));
        HIPCHK(hipMemsetAsync(in.qC.ptr, 0, (size_t)(in.ldqc * pp), st));
        hipLaunchKernelGGL(k_fp8_scales, dim3((unsigned)((pp + 3) / 4)), dim3(256), 0, st, Xh, ldx, np, pp,
                           in.qs.as<float>());
        hipLaunchKernelGGL(k_to_fp8, dim3(4096), dim3(256), 0, st, Xh, ldx, in.qs.as<float>(), in.qC.as<uint8_t>(),
                           in.ldqc, in.qR.as<uint8_t>(), in.ldqr, np, pp);
        in.cst.ensure(sizeof(float) * (size_t)ldp);
        hipLaunchKernelGGL(k_to_f32, dim3(64), dim3(256), 0, st, in.c64.as<double>(), in.cst.as<float>(), ldp);
    } else {
        in.cst.ensure(sizeof(double) * (size_t)ldp);
        HIPCHK(hipMemcpyAsync(in.cst.ptr, in.c64.ptr, sizeof(double) * (size_t)ldp, hipMemcpyDeviceToDevice, st));
    }
    HIPCHK(hipGetLastError());
    // ||y||^2 on the host (one small copy)
    std::vector<double> hy((size_t)n);
    HIPCHK(hipMemcpyAsync(hy.data(), in.y64.ptr, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double yy = 0.0;
    for (double v : hy) yy += v * v;
    in.yy = yy;
    ctx->has_data = true;
}

}  // namespace l0l2
