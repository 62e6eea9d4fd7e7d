// Internal declarations shared by the libri HIP sources (gfx950 only).
#pragma once
#include <functional>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/ri.h"

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));
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

// Value of v in lane src, for every lane of the wave.
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// Lower Cholesky of a 64 x 64 block and the inverse of its factor on one
// wave (the workgroup is exactly 64 lanes), with no waits on other waves.
// S[64][65] in LDS holds the block on entry (row-major; rows and columns at
// or beyond nb set to the identity by the caller; only the lower triangle is
// read) and the factor L (zero above the diagonal) on exit.
// - Factor, right-looking: lane r keeps row r in registers.  At step j the
//   pivot comes from lane j, every lane forms its L[r][j] and writes it to an
//   LDS column, and the trailing update a[c] -= L[r][j] L[c][j] (r >= c)
//   reads that column back as broadcast loads, 16 entries ahead of their use.
// - Inverse, forward substitution: lane c forms column c of X = L^{-1},
//   X[r][c] = (delta_rc - sum_{k<r} L[r][k] X[k][c]) / L[r][r], reading the
//   rows of L as broadcast loads, and passes it to store(r, c, value) (row r
//   across lanes is contiguous).
// A pivot that is not positive is reported through bad(j) and replaced by 1.
// Each pivot's reciprocal is formed once (hardware estimate and two Newton
// steps, within an ulp of 1/piv) and multiplies instead of dividing, which
// keeps the fully unrolled steps free of the division sequence.
template <class Bad, class Store>
__device__ __forceinline__ void chol_inv64_wave(double (*S)[65], int nb, Bad bad, Store store) {
    const int lane = threadIdx.x & 63;
    __shared__ double rdiag[64];
    __shared__ double col[64];
    double a[64];
    int first_bad = 64;   // branch-free inside the unrolled steps; reported once
#pragma unroll
    for (int c = 0; c < 64; ++c) a[c] = S[lane][c];
#pragma clang loop unroll(full)
    for (int j = 0; j < 64; ++j) {
        const double d = lane_bcast(a[j], j);
        first_bad = (j < nb && !(d > 0.0) && first_bad == 64) ? j : first_bad;
        const double piv = sqrt(d > 0.0 ? d : 1.0);
        double rp = __builtin_amdgcn_rcp(piv);
        rp = fma(rp, fma(-piv, rp, 1.0), rp);
        rp = fma(rp, fma(-piv, rp, 1.0), rp);
        rdiag[j] = rp;   // every lane writes the same value
        a[j] = lane > j ? a[j] * rp : (lane == j ? piv : 0.0);
        col[lane] = a[j];
        __syncthreads();
        // column j read back 16 entries at a time ahead of their updates
#pragma unroll
        for (int c0 = j + 1; c0 < 64; c0 += 16) {
            double l[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) l[t] = c0 + t < 64 ? col[c0 + t] : 0.0;
#pragma unroll
            for (int t = 0; t < 16; ++t)
                if (c0 + t < 64 && lane >= c0 + t) a[c0 + t] -= a[j] * l[t];
        }
        __syncthreads();
    }
    if (lane == 0 && first_bad < 64) bad(first_bad);
#pragma unroll
    for (int c = 0; c < 64; ++c) S[lane][c] = c <= lane ? a[c] : 0.0;
    __syncthreads();
    // row r of L read 16 entries at a time ahead of its products, into four
    // partial sums (independent chains)
    double x[64];
#pragma clang loop unroll(full)
    for (int r = 0; r < 64; ++r) {
        double v[4] = {r == lane ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < r; k0 += 16) {
            double l[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) l[t] = k0 + t < r ? S[r][k0 + t] : 0.0;
#pragma unroll
            for (int t = 0; t < 16; ++t)
                if (k0 + t < r) v[t & 3] -= l[t] * x[k0 + t];
        }
        x[r] = ((v[0] + v[1]) + (v[2] + v[3])) * rdiag[r];
        store(r, lane, x[r]);
    }
}

// ------------------------------------------------------------ launch helpers
namespace ri {

// GEMM C = alpha op(A) op(B) + beta C over a batch (row-major, FP64 MFMA).
// tri: 0 general; 1 op(A) lower triangular; 2 op(A) upper triangular;
// 3 op(B) upper triangular.
// lowerC: skip 64x64 tiles of C strictly above the diagonal.
hipError_t gemm_f64(bool ta, bool tb, int M, int N, int K, double alpha,
                    const double* A, int64_t lda, int64_t sA,
                    const double* B, int64_t ldb, int64_t sB, double beta,
                    double* C, int64_t ldc, int64_t sC, int batch, int tri, int lowerC,
                    hipStream_t s);

// In-place Cholesky A = L L^T (lower; upper triangle zeroed) of an n x n
// matrix, plus Linv = L^{-1} when Linv != nullptr.  dwork >= ceil(n/64)*4096
// doubles.  The first non-positive pivot index is atomically min-ed into
// *d_bad (device int, caller initialises it to INT_MAX).  block_done(k), if
// given, is called once block column k of L (rows k*64 onward) and its
// diagonal-block inverse in dwork are enqueued as final on s, before the
// trailing update of step k.
hipError_t cholesky_inv(double* A, int n, int64_t lda, double* Linv, int64_t ldi,
                        double* dwork, int* d_bad, hipStream_t s,
                        const std::function<hipError_t(int)>& block_done = nullptr);

// Linv = L^{-1} from the factor and its diagonal-block inverses (as left by
// cholesky_inv with Linv == nullptr).
hipError_t tri_inverse(const double* L, int n, int64_t lda, const double* Dinv, double* Linv, int64_t ldi,
                       hipStream_t s);
// The same in parts, for callers that spread the launches out: begin sets
// Linv to the identity, then steps k0 .. k1-1 (of ceil(n/64)) run in order,
// all on one stream.
hipError_t tri_inverse_begin(double* Linv, int n, int64_t ldi, hipStream_t s);
hipError_t tri_inverse_steps(const double* L, int n, int64_t lda, const double* Dinv, double* Linv, int64_t ldi,
                             int k0, int k1, hipStream_t s);

hipError_t fill(double* p, double v, int64_t n, hipStream_t s);
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
// max |x_i| into *out; red: scratch of 256 doubles
hipError_t max_abs(const double* x, int64_t n, double* out, double* red, hipStream_t s);
hipError_t copy(double* dst, const double* src, int64_t n, hipStream_t s);
hipError_t widen(const float* x, double* y, int64_t n, hipStream_t s);   // y = (double) x

}  // namespace ri

#define RI_TRY(expr)                                   \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return _e;               \
    } while (0)
