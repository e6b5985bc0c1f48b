// Device-side closed forms of the method and MFMA helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace l0l2 {

enum : uint8_t { CODE_FREE = 0, CODE_FIX0 = 1, CODE_FIX1 = 2 };

// The scalars of MethodParams in the arithmetic type T of the sweep.  When rho
// is a power of two, x / rho and x * (1 / rho) are the same correctly rounded
// number (both scale x by an exact power of two), so the update multiplies by
// inv_rho instead of dividing (rho_pow2 set).
template <class T>
struct DevParams {
    T M, rho, inv_rho;
    T a_plus_s, ridge, thr_free, thr_free_M;
    int free_quad, rho_pow2;
};

// x / rho, by the exact reciprocal when rho is a power of two.
template <class T>
__device__ __forceinline__ T div_rho(T x, const DevParams<T> &q) {
    return q.rho_pow2 ? x * q.inv_rho : x / q.rho;
}

template <class T>
__device__ __forceinline__ T clip_box(T x, T m) {
    return x > m ? m : (x < -m ? -m : x);
}

// beta-update of eq. (minbetalower): the proximal map of psi_i plus the box.
// F0 -> 0; F1 -> ridge shrink then clip; free coordinate with sqrt(l0/l2) <= M ->
// ridge shrink beyond |bt| >= a + s, box soft threshold T(bt; a, M) below; free
// coordinate with sqrt(l0/l2) > M -> T(bt; l0/(M rho) + l2 M / rho, M).
template <class T>
__device__ __forceinline__ T prox_beta(T bt, uint8_t code, const DevParams<T> &q) {
    if (code == CODE_FIX0) return T(0);
    T ab = fabs(bt);
    if (code == CODE_FIX1 || (q.free_quad && ab >= q.a_plus_s)) return clip_box(q.ridge * bt, q.M);
    T sg = bt > T(0) ? T(1) : (bt < T(0) ? T(-1) : T(0));
    if (ab <= q.thr_free) return T(0);
    if (ab <= q.thr_free_M) return (ab - q.thr_free) * sg;
    return q.M * sg;
}

// psi_i(beta) of eq. (psi) for an iterate inside the box (FP64).
__device__ __forceinline__ double psi_val(double beta, uint8_t code, double l0, double l2, double s,
                                          int free_quad, double psi_lin) {
    if (code == CODE_FIX0) return beta == 0.0 ? 0.0 : INFINITY;
    double ab = fabs(beta);
    if (code == CODE_FIX1) return l0 + l2 * beta * beta;
    if (free_quad) {
        if (ab >= s) return l0 + l2 * beta * beta;
        return psi_lin * ab;
    }
    return psi_lin * ab;
}

// z_i of App. A.1 for a given beta_i (FP64).
__device__ __forceinline__ double z_of(double beta, uint8_t code, double s, double M, int free_quad) {
    if (code == CODE_FIX0) return 0.0;
    if (code == CODE_FIX1) return 1.0;
    double ab = fabs(beta);
    if (free_quad) return ab >= s ? 1.0 : ab / s;
    return ab / M;
}

// Upper bound of nu_i(|X_i^T r|) (eq. nudef) given the computed |g| and its
// a-priori error e: nu is nondecreasing, so it is taken at x = (|g| + e)(1 + 4u)
// and raised by gamma_4 times the magnitude of its terms.
__device__ __forceinline__ double nu_upper(double absg, double e, uint8_t code, double l0, double l2,
                                           double M, double two_M_l2, double four_l2, double l2_M2,
                                           int free_quad) {
    const double u = 1.1102230246251565e-16;  // 2^-53
    const double g4 = 4.0 * u / (1.0 - 4.0 * u);
    if (code == CODE_FIX0) return 0.0;
    double x = (absg + e) * (1.0 + 4.0 * u);
    double val, mag;
    if (code == CODE_FIX1 || free_quad) {
        if (x <= two_M_l2) {
            val = x * x / four_l2 - l0;
            mag = x * x / four_l2 + l0;
        } else {
            val = M * x - l0 - l2_M2;
            mag = M * x + l0 + l2_M2;
        }
    } else {
        val = M * x - l0 - l2_M2;
        mag = M * x + l0 + l2_M2;
    }
    val += g4 * mag;
    if (code == CODE_FREE && val < 0.0) val = 0.0;
    return val;
}

// nu_i(|g|) of eq. (nudef) in plain FP64 (no rounding allowance): the value the
// gap estimate uses to decide whether a node can have converged.
__device__ __forceinline__ double nu_plain(double absg, uint8_t code, double l0, double l2, double M,
                                           double two_M_l2, double four_l2, double l2_M2, int free_quad) {
    if (code == CODE_FIX0) return 0.0;
    double val;
    if ((code == CODE_FIX1 || free_quad) && absg <= two_M_l2) val = absg * absg / four_l2 - l0;
    else val = M * absg - l0 - l2_M2;
    if (code == CODE_FREE && val < 0.0) val = 0.0;
    return val;
}

__device__ __forceinline__ double gamma_k(double k) {
    const double u = 1.1102230246251565e-16;
    return k * u / (1.0 - k * u);
}

// ---------------------------------------------------------------------------
// MFMA wrappers (wave64).  For both 16x16 shapes lane l supplies A[l%16][k] and
// B[k][l%16] for its k slot; the 4 accumulators of lane l hold column l%16 of D
// at rows 4*(l/16)+v (f32 variants) or l/16 + 4*v (f64 variant).
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <class T> struct Acc;
template <> struct Acc<float> { typedef f32x4 type; };
template <> struct Acc<double> { typedef f64x4 type; };

// Row of accumulator v held by lane l (column is l % 16).
template <class T> __device__ __forceinline__ int acc_row(int lane, int v);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <> __device__ __forceinline__ int acc_row<double>(int lane, int v) { return (lane >> 4) + 4 * v; }

template <class T> struct Vec4;
template <> struct Vec4<float> { typedef float4 type; };
template <> struct Vec4<double> { typedef double4 type; };

template <class T>
__device__ __forceinline__ void load4(const T *p, T out[4]) {
    typedef typename Vec4<T>::type V;
    V v = *reinterpret_cast<const V *>(p);
    out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
}

}  // namespace l0l2
