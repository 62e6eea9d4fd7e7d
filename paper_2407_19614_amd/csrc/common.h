// Internal declarations shared by the libri HIP sources (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/ri.h"

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
// LDS destination operand of __builtin_amdgcn_global_load_lds
typedef __attribute__((address_space(3))) void* lds_void_t;

#define RI_PI 3.14159265358979323846

// v_mfma_f64_16x16x4_f64: D(16x16) += A(16x4) B(4x16).
// Lane l supplies A[l%16][l/16] and B[l/16][l%16]; it receives
// D[4*r + l/16][l%16] in element r of the result.
__device__ __forceinline__ d4_t mfma_f64(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  This bijection maps the hardware order onto a logical order in which
// each XCD receives one contiguous run of logical workgroup ids, so that
// neighbouring logical work (sharing operands) shares an L2.
__device__ __forceinline__ int xcd_remap(int L, int W) {
    const int q = W >> 3, r = W & 7, x = L & 7, s = L >> 3;
    return x * q + min(x, r) + s;
}

__device__ __forceinline__ double norm_s(double a) {
    // (2a/pi)^{3/4}
    return pow(2.0 * a / RI_PI, 0.75);
}

// Boys function F0(t) = int_0^1 exp(-t u^2) du.
__device__ __forceinline__ double boys_f0(double t) {
    if (t < 1e-4) {
        // 1 - t/3 + t^2/10 - t^3/42 + t^4/216
        return 1.0 + t * (-1.0 / 3.0 + t * (1.0 / 10.0 + t * (-1.0 / 42.0 + t * (1.0 / 216.0))));
    }
    double s = sqrt(t);
    return 0.88622692545275801365 * erf(s) / s;   // sqrt(pi)/2
}

// Boys function F1(t) = int_0^1 u^2 exp(-t u^2) du.  For t < 1 the series
// F1 = exp(-t) sum_k (2t)^k / (3*5*...*(2k+3)) (all terms positive);
// otherwise the downward relation F1 = (F0 - exp(-t)) / (2t).
__device__ __forceinline__ double boys_f1(double t) {
    double e = exp(-t);
    if (t < 1.0) {
        double term = 1.0 / 3.0, sum = term;
        double x = 2.0 * t;
        #pragma unroll 1
        for (int k = 1; k < 40; ++k) {
            term *= x / (2.0 * k + 3.0);
            sum += term;
            if (term < 1e-17 * sum) break;
        }
        return e * sum;
    }
    return (boys_f0(t) - e) / (2.0 * t);
}

// Lower Cholesky of an nb x nb (nb <= 64) block held in LDS as L[64][65]
// (rows/columns beyond nb set to the identity by the caller), in place on
// and below the diagonal, and its inverse, written through store(i, c, value)
// for all 64 x 64 entries (zero above the diagonal, identity beyond nb).  A
// workgroup of NT threads (NT / 64 waves) runs it: at step j the pivot and
// column j are finished, row j of the inverse is scaled, and then every wave
// takes rows i > j of both the trailing Cholesky update and the forward
// elimination X_i -= L_ij X_j, one column per lane, so each step is two
// barriers of uniform work.  A pivot that is not positive is reported through
// bad(j) and replaced by 1.
template <int NT, class Bad, class Store>
__device__ __forceinline__ void potrf_inv_block64(double (*L)[65], int nb, Bad bad, Store store) {
    static_assert(NT % 64 == 0, "whole waves");
    constexpr int NW = NT / 64;
    __shared__ double X[64][65];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int i = wv; i < 64; i += NW) X[i][lane] = i == lane ? 1.0 : 0.0;
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        const double d = L[j][j];
        const double piv = sqrt(d > 0.0 ? d : 1.0);
        if (wv == 0) {
            if (lane == 0 && !(d > 0.0)) bad(j);
            if (lane > j && lane < nb) L[lane][j] /= piv;      // column j of the factor
            if (lane <= j) X[j][lane] /= piv;                   // row j of the inverse
        }
        __syncthreads();
        if (t == 0) L[j][j] = piv;
        const double lcj = lane > j ? L[lane][j] : 0.0, xjc = X[j][lane];
        for (int i = j + 1 + wv; i < nb; i += NW) {
            const double lij = L[i][j];
            if (lane > j && lane <= i) L[i][lane] -= lij * lcj;
            if (lane <= j) X[i][lane] -= lij * xjc;
        }
        __syncthreads();
    }
    for (int i = wv; i < 64; i += NW) store(i, lane, X[i][lane]);
}

// ------------------------------------------------------------ launch helpers
namespace ri {

// GEMM C = alpha op(A) op(B) + beta C over a batch (row-major, FP64 MFMA).
// tri: 0 general; 1 op(A) lower triangular; 2 op(A) upper triangular.
// lowerC: skip 64x64 tiles of C strictly above the diagonal.
hipError_t gemm_f64(bool ta, bool tb, int M, int N, int K, double alpha,
                    const double* A, int64_t lda, int64_t sA,
                    const double* B, int64_t ldb, int64_t sB, double beta,
                    double* C, int64_t ldc, int64_t sC, int batch, int tri, int lowerC,
                    hipStream_t s);

// In-place Cholesky A = L L^T (lower; upper triangle zeroed) of an n x n
// matrix, plus Linv = L^{-1} when Linv != nullptr.  dwork >= ceil(n/64)*4096
// doubles.  The first non-positive pivot index is atomically min-ed into
// *d_bad (device int, caller initialises it to INT_MAX).
hipError_t cholesky_inv(double* A, int n, int64_t lda, double* Linv, int64_t ldi,
                        double* dwork, int* d_bad, hipStream_t s);

// In place B <- L^{-1} B for lower L (n x n) whose 64 x 64 diagonal-block
// inverses are in Dinv (as left by cholesky_inv); B has ncols columns.
hipError_t trsm_lower_inplace(const double* L, int n, int64_t lda, const double* Dinv, double* B, int ncols,
                              int64_t ldb, hipStream_t s);
hipError_t fill(double* p, double v, int64_t n, hipStream_t s);
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t set_identity(double* p, int n, int64_t ld, hipStream_t s);
// out[k] = sum_i x[i] * y[i] for one pair of vectors, accumulated as
// out[slot] (single block per call, deterministic).
hipError_t dot(const double* x, const double* y, int64_t n, double* out, hipStream_t s);
// max |x_i| into *out; red: scratch of 256 doubles
hipError_t max_abs(const double* x, int64_t n, double* out, double* red, hipStream_t s);
hipError_t axpby(double* y, const double* x, double a, double b, int64_t n, hipStream_t s); // y = a x + b y
hipError_t copy(double* dst, const double* src, int64_t n, hipStream_t s);
hipError_t widen(const float* x, double* y, int64_t n, hipStream_t s);   // y = (double) x

}  // namespace ri

#define RI_TRY(expr)                                   \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return _e;               \
    } while (0)
