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
    // from t = 40 on, erf(sqrt t) is 1 in double precision (erfc < 2e-19)
    if (t >= 40.0) return 0.88622692545275801365 / s;
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
// read) and the factor L (zero above the diagonal) on exit; X = L^{-1}
// (lower, zero above the diagonal) is passed entry by entry to
// store(row, column, value).  A pivot that is not positive is reported
// through bad(j) (the first one) and replaced by 1.
// The work runs in 16 x 16 blocks.  For each diagonal block k: its 16 x 16
// factor and the inverse of that factor by lanes 0-15 (lane r keeps row r;
// broadcasts by lane reads; each pivot's reciprocal from the hardware
// estimate and two Newton steps), and then the panel blocks
// L_ik = A_ik (L_kk^{-1})^T and the trailing updates A_ij -= L_ik L_jk^T on
// FP64 MFMA with operands read from S.  The latency chains are 16 steps
// long instead of 64.  Then L^{-1} by block forward substitution,
// X_ij = -L_ii^{-1} sum_{j<=k<i} L_ik X_kj, also on MFMA, with the X blocks
// in registers: an accumulator tile (element q of lane (c, g) holds row
// 4q + g of column c) is already the B operand of the next product over its
// 16 rows.
template <class Bad, class Store>
__device__ __forceinline__ void chol_inv64_blocked(double (*S)[65], int nb, Bad bad, Store store) {
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    __shared__ double Di[4][16][17];   // inverses of the diagonal 16 x 16 factors
    int first_bad = 64;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const int o = 16 * kb;
        // factor of the diagonal block: lane r keeps its row
        double a[16];
        double rd = 1.0;
#pragma unroll
        for (int c = 0; c < 16; ++c) a[c] = (lane < 16 && c <= lane) ? S[o + r][o + c] : 0.0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const double d = lane_bcast(a[j], j);
            first_bad = (o + j < nb && !(d > 0.0) && first_bad == 64) ? o + j : first_bad;
            const double piv = sqrt(d > 0.0 ? d : 1.0);
            double rp = __builtin_amdgcn_rcp(piv);
            rp = fma(rp, fma(-piv, rp, 1.0), rp);
            rp = fma(rp, fma(-piv, rp, 1.0), rp);
            rd = lane == j ? rp : rd;
            a[j] = lane > j ? a[j] * rp : (lane == j ? piv : 0.0);
#pragma unroll
            for (int c = j + 1; c < 16; ++c) a[c] = fma(-a[j], lane_bcast(a[j], c), a[c]);
        }
        if (lane < 16) {
#pragma unroll
            for (int c = 0; c < 16; ++c) S[o + r][o + c] = c <= lane ? a[c] : 0.0;
        }
        // inverse of the diagonal factor: lane c forms its column
        {
            double x[16];
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) {
                double v = rr == lane ? 1.0 : 0.0;
#pragma unroll
                for (int k = 0; k < rr; ++k) v -= lane_bcast(a[k], rr) * x[k];
                x[rr] = v * lane_bcast(rd, rr);
                if (lane < 16) Di[kb][rr][lane] = x[rr];
            }
        }
        __syncthreads();
        // panel: L_ik = A_ik (L_kk^{-1})^T, B[k][c] = Di[c][k]; the blocks are
        // independent, so their MFMA chains interleave, and each block reads
        // only the entries it rewrites (one wave: program order suffices)
        {
            d4_t acc[3];
#pragma unroll
            for (int ib = kb + 1; ib < 4; ++ib) acc[ib - kb - 1] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const double bk = Di[kb][r][4 * s4 + g];
#pragma unroll
                for (int ib = kb + 1; ib < 4; ++ib)
                    acc[ib - kb - 1] = mfma_f64(S[16 * ib + r][o + 4 * s4 + g], bk, acc[ib - kb - 1]);
            }
#pragma unroll
            for (int ib = kb + 1; ib < 4; ++ib)
#pragma unroll
                for (int q = 0; q < 4; ++q) S[16 * ib + 4 * q + g][o + r] = acc[ib - kb - 1][q];
        }
        __syncthreads();
        // trailing: A_ij -= L_ik L_jk^T, B[k][c] = L_jk[c][k]; the blocks read
        // the panel and write disjoint blocks, so they interleave too
        {
            constexpr int NTB = 6;   // at most 6 blocks (k = 0)
            d4_t acc[NTB];
            int n = 0;
#pragma unroll
            for (int jb = kb + 1; jb < 4; ++jb)
#pragma unroll
                for (int ib = jb; ib < 4; ++ib, ++n)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[n][q] = S[16 * ib + 4 * q + g][16 * jb + r];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                double pj[4];
#pragma unroll
                for (int b = kb + 1; b < 4; ++b) pj[b] = S[16 * b + r][o + 4 * s4 + g];
                n = 0;
#pragma unroll
                for (int jb = kb + 1; jb < 4; ++jb)
#pragma unroll
                    for (int ib = jb; ib < 4; ++ib, ++n) acc[n] = mfma_f64(-pj[ib], pj[jb], acc[n]);
            }
            n = 0;
#pragma unroll
            for (int jb = kb + 1; jb < 4; ++jb)
#pragma unroll
                for (int ib = jb; ib < 4; ++ib, ++n)
#pragma unroll
                    for (int q = 0; q < 4; ++q) S[16 * ib + 4 * q + g][16 * jb + r] = acc[n][q];
        }
        __syncthreads();
    }
    if (lane == 0 && first_bad < 64) bad(first_bad);
    // zero above the diagonal (the diagonal blocks were written lower only)
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int jb = ib + 1; jb < 4; ++jb)
#pragma unroll
            for (int q = 0; q < 4; ++q) S[16 * ib + 4 * q + g][16 * jb + r] = 0.0;
    __syncthreads();
    // X = L^{-1}: X_ii = Di[i]; X_ij = -Di[i] sum_{j<=k<i} L_ik X_kj
    d4_t X[4][4];
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int q = 0; q < 4; ++q) X[ib][ib][q] = Di[ib][4 * q + g][r];
    // block row i at a time; its blocks j < i are independent chains
#pragma unroll
    for (int ib = 1; ib < 4; ++ib) {
        d4_t t[3];
#pragma unroll
        for (int jb = 0; jb < ib; ++jb) t[jb] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kb = 0; kb < ib; ++kb)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const double l = S[16 * ib + r][16 * kb + 4 * s4 + g];
#pragma unroll
                for (int jb = 0; jb <= kb; ++jb) t[jb] = mfma_f64(l, X[kb][jb][s4], t[jb]);
            }
#pragma unroll
        for (int jb = 0; jb < ib; ++jb) X[ib][jb] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const double di = -Di[ib][r][4 * s4 + g];
#pragma unroll
            for (int jb = 0; jb < ib; ++jb) X[ib][jb] = mfma_f64(di, t[jb][s4], X[ib][jb]);
        }
    }
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int q = 0; q < 4; ++q) store(16 * ib + 4 * q + g, 16 * jb + r, jb <= ib ? X[ib][jb][q] : 0.0);
}

// ------------------------------------------------------------ launch helpers
namespace ri {

// GEMM C = alpha op(A) op(B) + beta C over a batch (row-major, FP64 MFMA).
// tri: 0 general; 1 op(A) lower triangular; 2 op(A) upper triangular;
// 3 op(B) upper triangular.
// lowerC: skip tiles of C strictly above the diagonal.
// tile: 0 picks 64- or 128-wide tiles from the shape; 64 or 128 forces one.
hipError_t gemm_f64(bool ta, bool tb, int M, int N, int K, double alpha,
                    const double* A, int64_t lda, int64_t sA,
                    const double* B, int64_t ldb, int64_t sB, double beta,
                    double* C, int64_t ldc, int64_t sC, int batch, int tri, int lowerC,
                    hipStream_t s, int tile = 0);

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
