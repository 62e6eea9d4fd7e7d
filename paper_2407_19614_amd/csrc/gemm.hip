// FP64 MFMA GEMM and the dense linear algebra built on it: blocked Cholesky
// with non-positive pivot detection and the triangular inverse.
#include "common.h"
#include "kernels.h"
#include <climits>
#include <functional>

namespace {

constexpr int BM = 64, BN = 64, BK = 16, LDP = BM + 1;

// 256 threads = 4 waves in a 2 x 2 arrangement; each wave owns a 32 x 32
// block of C as 2 x 2 MFMA 16x16 tiles.  Tiles of A and B are staged through
// LDS in k-major order so that the 16 lanes reading one fragment row touch
// consecutive addresses.  Global loads for the next k-slice are issued before
// the MFMAs of the current one.
template <bool TA, bool TB>
__device__ __forceinline__ void gemm_tile64(int M, int N, int K, double alpha, const double* __restrict__ A,
                                            int64_t lda, const double* __restrict__ B, int64_t ldb, double beta,
                                            double* __restrict__ C, int64_t ldc, int tri, int m0, int n0,
                                            bool sym = false) {
    __shared__ double As[BK][LDP];
    __shared__ double Bs[BK][LDP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;

    int kbeg = 0, kend = K;
    if (tri == 1) kend = min(K, m0 + BM);
    if (tri == 2) kbeg = (m0 / BK) * BK;
    if (tri == 3) kend = min(K, n0 + BN);

    double ra[4], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int m, k;
            if (!TA) { k = tid & 15; m = (tid >> 4) + 16 * r; }
            else     { m = tid & 63; k = (tid >> 6) + 4 * r; }
            int gm = m0 + m, gk = k0 + k;
            double v = 0.0;
            if (gm < M && gk < kend)
                v = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
            ra[r] = v;
            int n, kb;
            if (!TB) { n = tid & 63; kb = (tid >> 6) + 4 * r; }
            else     { kb = tid & 15; n = (tid >> 4) + 16 * r; }
            int gn = n0 + n, gkb = k0 + kb;
            double w = 0.0;
            if (gn < N && gkb < kend)
                w = TB ? B[(int64_t)gn * ldb + gkb] : B[(int64_t)gkb * ldb + gn];
            rb[r] = w;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int m, k;
            if (!TA) { k = tid & 15; m = (tid >> 4) + 16 * r; }
            else     { m = tid & 63; k = (tid >> 6) + 4 * r; }
            As[k][m] = ra[r];
            int n, kb;
            if (!TB) { n = tid & 63; kb = (tid >> 6) + 4 * r; }
            else     { kb = tid & 15; n = (tid >> 4) + 16 * r; }
            Bs[kb][n] = rb[r];
        }
    };

    d4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

    const int li = lane & 15, lk = lane >> 4;
    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();
        store();
        __syncthreads();
        if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double a0 = As[kk + lk][wm + li], a1 = As[kk + lk][wm + 16 + li];
            double b0 = Bs[kk + lk][wn + li], b1 = Bs[kk + lk][wn + 16 + li];
            acc[0][0] = mfma_f64(a0, b0, acc[0][0]);
            acc[0][1] = mfma_f64(a0, b1, acc[0][1]);
            acc[1][0] = mfma_f64(a1, b0, acc[1][0]);
            acc[1][1] = mfma_f64(a1, b1, acc[1][1]);
        }
    }
    // With beta != 0 every C value of the tile is loaded before the first
    // store (from addresses clamped into the matrix, so without branches):
    // loads placed after stores to C would each wait out a full memory
    // latency, since the compiler cannot prove the addresses distinct.
    double cv[2][2][4];
    if (beta != 0.0) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gm = min(m0 + wm + 16 * i + 4 * r + lk, M - 1), gn = min(n0 + wn + 16 * j + li, N - 1);
                    cv[i][j][r] = C[(int64_t)gm * ldc + gn];
                }
    }
    // all results before the first store: stores count against the same
    // wait counter as the loads
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                cv[i][j][r] = alpha * acc[i][j][r] + (beta != 0.0 ? beta * cv[i][j][r] : 0.0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int gm = m0 + wm + 16 * i + 4 * r + lk, gn = n0 + wn + 16 * j + li;
                if (gm < M && gn < N && !(sym && gm > gn)) {
                    C[(int64_t)gm * ldc + gn] = cv[i][j][r];
                    if (sym && gm != gn) C[(int64_t)gn * ldc + gm] = cv[i][j][r];
                }
            }
}

// upper tile t (row-major over I <= J) of a t x t tiling
__device__ __forceinline__ void upper_tile(int t, int nt, int& I, int& J) {
    int i = 0, rem = t;
    while (rem >= nt - i) {
        rem -= nt - i;
        ++i;
    }
    I = i;
    J = i + rem;
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f64_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, int64_t lda, int64_t sA,
    const double* __restrict__ B, int64_t ldb, int64_t sB, double beta, double* __restrict__ C,
    int64_t ldc, int64_t sC, int tri, int lowerC) {
    const int gx = gridDim.x, gy = gridDim.y;
    const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int L = tri != 0 ? lin : xcd_remap(lin, gx * gy * gridDim.z);   // as in the 128-wide form
    const int bx = L % gx, by = (L / gx) % gy, bz = L / (gx * gy);
    const int m0 = by * BM, n0 = bx * BN;
    if (lowerC && n0 > m0 + BM - 1) return;
    gemm_tile64<TA, TB>(M, N, K, alpha, A + (int64_t)bz * sA, lda, B + (int64_t)bz * sB, ldb, beta,
                        C + (int64_t)bz * sC, ldc, tri, m0, n0);
}

// Grouped GEMM: problem g owns tiles prefix[g] .. prefix[g+1]-1 (row-major
// over its 64 x 64 tiles); a problem whose `active` flag is 0 is skipped.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_grouped_kernel(const ri::GemmDesc* d, const int* prefix, int n) {
    int g, loc;
    ri::decode_item(prefix, n, blockIdx.x, g, loc);
    const ri::GemmDesc& p = d[g];
    if (p.active && !*p.active) return;
    const int tn = (p.N + BN - 1) / BN;
    int I = loc / tn, J = loc % tn;
    if (p.sym) upper_tile(loc, tn, I, J);
    gemm_tile64<TA, TB>(p.M, p.N, p.K, p.alpha, p.A, p.lda, p.B, p.ldb, p.beta, p.C, p.ldc, p.tri, I * BM, J * BN,
                        p.sym != 0);
}

// 128 x 128 variant: 4 waves in 2 x 2, each owning 64 x 64 of C as 4 x 4 MFMA
// tiles (64 FP64 accumulators per lane).  Same staging scheme as above.
template <bool TA, bool TB, int BK = ::BK>
__device__ __forceinline__ void gemm_tile128(int M, int N, int K, double alpha, const double* __restrict__ A,
                                             int64_t lda, const double* __restrict__ B, int64_t ldb, double beta,
                                             double* __restrict__ C, int64_t ldc, int tri, int m0, int n0,
                                             bool sym = false) {
    constexpr int TM = 128, LD = TM + 1, R = BK / 2;   // R: elements of each operand per thread per slice
    __shared__ double As[BK][LD];
    __shared__ double Bs[BK][LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    int kbeg = 0, kend = K;
    if (tri == 1) kend = min(K, m0 + TM);
    if (tri == 2) kbeg = (m0 / BK) * BK;
    if (tri == 3) kend = min(K, n0 + TM);
    double ra[R], rb[R];
    // thread tid covers (k-major) k = tid % BK, m = tid / BK + (256 / BK) r, or
    // (m-major) m = tid % 128, k = tid / 128 + 2 r
    constexpr int MS = 256 / BK;
    auto load = [&](int k0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int m, k;
            if (!TA) { k = tid % BK; m = tid / BK + MS * r; }
            else     { m = tid & 127; k = (tid >> 7) + 2 * r; }
            int gm = m0 + m, gk = k0 + k;
            ra[r] = (gm < M && gk < kend) ? (TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk]) : 0.0;
            int n, kb;
            if (!TB) { n = tid & 127; kb = (tid >> 7) + 2 * r; }
            else     { kb = tid % BK; n = tid / BK + MS * r; }
            int gn = n0 + n, gkb = k0 + kb;
            rb[r] = (gn < N && gkb < kend) ? (TB ? B[(int64_t)gn * ldb + gkb] : B[(int64_t)gkb * ldb + gn]) : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int m, k;
            if (!TA) { k = tid % BK; m = tid / BK + MS * r; }
            else     { m = tid & 127; k = (tid >> 7) + 2 * r; }
            As[k][m] = ra[r];
            int n, kb;
            if (!TB) { n = tid & 127; kb = (tid >> 7) + 2 * r; }
            else     { kb = tid % BK; n = tid / BK + MS * r; }
            Bs[kb][n] = rb[r];
        }
    };
    d4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
    const int li = lane & 15, lk = lane >> 4;
    if (kbeg < kend) load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();
        store();
        __syncthreads();
        if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk + lk][wm + 16 * i + li];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk + lk][wn + 16 * j + li];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
        }
    }
    // Epilogue by 16-row slices: with beta != 0 the slice's 16 C values are
    // loaded (clamped addresses, no branches) before its stores, so each
    // slice waits out one memory latency rather than one per element.
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double cv[4][4];
        if (beta != 0.0) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int gm = min(m0 + wm + 16 * i + 4 * r + lk, M - 1), gn = min(n0 + wn + 16 * j + li, N - 1);
                    cv[j][r] = C[(int64_t)gm * ldc + gn];
                }
        }
        // all 16 results before the first store: stores count against the
        // same wait counter as the loads
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) cv[j][r] = alpha * acc[i][j][r] + (beta != 0.0 ? beta * cv[j][r] : 0.0);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int gm = m0 + wm + 16 * i + 4 * r + lk, gn = n0 + wn + 16 * j + li;
                if (gm < M && gn < N && !(sym && gm > gn)) {
                    C[(int64_t)gm * ldc + gn] = cv[j][r];
                    if (sym && gm != gn) C[(int64_t)gn * ldc + gm] = cv[j][r];
                }
            }
    }
}

template <bool TA, bool TB, int SBK = BK>
__global__ __launch_bounds__(256, 2) void gemm_f64_128_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, int64_t lda, int64_t sA,
    const double* __restrict__ B, int64_t ldb, int64_t sB, double beta, double* __restrict__ C,
    int64_t ldc, int64_t sC, int tri, int lowerC) {
    constexpr int TM = 128, TN = 128;
    const int gx = gridDim.x, gy = gridDim.y;
    // Contiguous runs of tiles per XCD keep shared operands in one L2, but with
    // a triangular operand the work per tile changes along the rows (or
    // columns), and with lowerC the number of live tiles per row does, so the
    // XCD holding one end would carry most of the work: there the tiles go
    // round-robin over the XCDs in launch order instead.
    const int lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int L = (tri != 0 || lowerC) ? lin : xcd_remap(lin, gx * gy * gridDim.z);
    const int bx = L % gx, by = (L / gx) % gy, bz = L / (gx * gy);
    const int m0 = by * TM, n0 = bx * TN;
    if (lowerC && n0 > m0 + TM - 1) return;
    gemm_tile128<TA, TB, SBK>(M, N, K, alpha, A + (int64_t)bz * sA, lda, B + (int64_t)bz * sB, ldb, beta,
                              C + (int64_t)bz * sC, ldc, tri, m0, n0);
}

// Grouped GEMM on 128 x 128 tiles: problem g owns tiles prefix[g] ..
// prefix[g+1]-1 (row-major over its tiles); inactive problems are skipped.
template <bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void gemm_grouped128_kernel(const ri::GemmDesc* d, const int* prefix, int n) {
    int g, loc;
    ri::decode_item(prefix, n, blockIdx.x, g, loc);
    const ri::GemmDesc& p = d[g];
    if (p.active && !*p.active) return;
    const int tn = (p.N + 127) / 128;
    int I = loc / tn, J = loc % tn;
    if (p.sym) upper_tile(loc, tn, I, J);
    gemm_tile128<TA, TB>(p.M, p.N, p.K, p.alpha, p.A, p.lda, p.B, p.ldb, p.beta, p.C, p.ldc, p.tri, I * 128, J * 128,
                         p.sym != 0);
}

// Factor one 64x64 diagonal block in place (lower Cholesky) and write the
// inverse of its factor to Dinv (64x64, lower, identity padding beyond n).
// One wave; rows are loaded and stored across lanes (coalesced).
__global__ __launch_bounds__(64) void potrf_diag_kernel(double* A, int n, int64_t lda, int kb, double* Dinv,
                                                         int* bad) {
    __shared__ double S[64][65];
    const int lane = threadIdx.x, o = kb * 64, nb = min(64, n - o);
    for (int r = 0; r < 64; ++r)
        S[r][lane] = (r < nb && lane < nb) ? A[(int64_t)(o + r) * lda + o + lane] : (r == lane ? 1.0 : 0.0);
    __syncthreads();
    chol_inv64_blocked(S, nb, [&](int j) { atomicMin(bad, o + j); }, [&](int i, int c, double v) { Dinv[i * 64 + c] = v; });
    __syncthreads();
    for (int r = 0; r < nb; ++r)
        if (lane < nb) A[(int64_t)(o + r) * lda + o + lane] = S[r][lane];
}

__global__ void zero_upper_kernel(double* A, int n, int64_t lda) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * n) return;
    int r = i / n, c = i % n;
    if (c > r) A[(int64_t)r * lda + c] = 0.0;
}

__global__ void fill_kernel(double* p, double v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void identity_kernel(double* p, int n, int64_t ld) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * n) return;
    int r = i / n, c = i % n;
    p[(int64_t)r * ld + c] = (r == c) ? 1.0 : 0.0;
}
__global__ void f32_to_f64_kernel(const float* x, double* y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}

__device__ double block_sum(double v) {
    __shared__ double sh[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}
__device__ double block_max(double v) {
    __shared__ double sh[16];
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o));
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, sh[i]);
    return r;
}

// max |x| in two stages: 256 workgroups over grid-stride shares, then one
__global__ __launch_bounds__(1024) void maxabs_kernel(const double* x, int64_t n, double* out) {
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s = fmax(s, fabs(x[i]));
    s = block_max(s);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Band of the factor in the leaf kernel's operand order: slot (k, d) of
// P (4096 doubles each, 4 slots per 64-row block k) holds Dinv_k for d = 0
// and -L_{k+d, k} (zero beyond row n) for d = 1..3, element
// ((4 q + t) 64 + l) 4 + u being entry (16 q + l % 16, 16 t + 4 u + l / 16)
// of the 64 x 64 block: lane l's four A operands of one 16 x 16 MFMA slice
// pass are contiguous, and the 64 lanes read 2 KB in one run.
__global__ void trsm_band_kernel(const double* __restrict__ L, int n, int64_t lda, const double* __restrict__ Dinv,
                                 double* __restrict__ P) {
    const int nb = (n + 63) / 64;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)nb * 4 * 4096) return;
    const int slot = (int)(e >> 12), k = slot >> 2, d = slot & 3, w = (int)(e & 4095);
    if (k + d >= nb) return;
    const int u = w & 3, l = (w >> 2) & 63, t = (w >> 8) & 3, q = w >> 10;
    const int row = 16 * q + (l & 15), col = 16 * t + 4 * u + (l >> 4);
    double v;
    if (d == 0) {
        v = Dinv[(int64_t)k * 4096 + row * 64 + col];
    } else {
        const int gr = 64 * (k + d) + row;
        v = gr < n ? -L[(int64_t)gr * lda + 64 * k + col] : 0.0;
    }
    P[e] = v;
}

// Leaf of the blocked forward substitution B <- L^{-1} B for n <= 64 NB rows,
// held in registers: each wave owns 16 columns of B (n x 16 as 4 NB MFMA
// accumulator tiles, zero beyond row n) and runs the 64-row block steps
// X_k = Dinv_k B_k, then B_m -= L_mk X_k for every block m below k, with
// FP64 MFMA, reading the band P (above) straight from memory: every wave
// reads the same slots, so they are cache hits.  The reduction index of each
// MFMA is k = 16 t + 4 s + g for lane group g and slice s: an accumulator
// tile in the C layout (element s of lane (c, g) holds row 4s + g of column
// c) is then already the B operand of the four slices over its 16 rows.
// The work runs in chunks of 16 MFMAs (one 16-deep slice t against the four
// 16-row tiles of one block, four independent accumulators), each chunk's
// 16 A values loaded one chunk ahead.  Dinv_k carries identity padding
// beyond the last row of a ragged final block and the band is zero there,
// so padded rows stay zero.  B is read and written once.
template <int NB>
__global__ __launch_bounds__(256, 2) void trsm_leaf_kernel(const double* __restrict__ P, double* __restrict__ B,
                                                           int n, int ncols, int64_t ldb) {
    constexpr int NT = 4 * NB;
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    const int c0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (c0 >= ncols) return;
    const int col = min(c0 + r, ncols - 1);
    d4_t acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * j + 4 * i + g;
            const double v = B[(int64_t)min(row, n - 1) * ldb + col];
            acc[j][i] = row < n ? v : 0.0;
        }
    // A values of chunk (kb, mb, t): block mb's four row tiles against the
    // 16-deep slice t of block kb, from band slot (kb, mb - kb).  Buffer
    // loads: the lane offset is fixed and the chunk's offset is a scalar, so
    // no vector address is formed (or kept) per chunk.
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(P), (short)0, NB * 4 * 4096 * 8, 0x00020000);
    const int voff = lane * 32;
    auto fetch = [&](int kb, int mb, int t, double (&a)[4][4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int so = ((kb * 4 + (mb - kb)) * 4096 + (4 * q + t) * 256) * 8;
            const d2_t lo = __builtin_bit_cast(d2_t, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, so, 0));
            const d2_t hi = __builtin_bit_cast(d2_t, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, so + 16, 0));
            a[q][0] = lo[0]; a[q][1] = lo[1]; a[q][2] = hi[0]; a[q][3] = hi[1];
        }
    };
    double cur[4][4], nxt[4][4];
    fetch(0, 0, 0, cur);
    d4_t x[4];
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int mb = kb; mb < NB; ++mb) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                int nkb = kb, nmb = mb, ntt = t + 1;
                if (ntt == 4) {
                    ntt = 0;
                    if (++nmb == NB) nmb = ++nkb;
                }
                if (nkb < NB) fetch(nkb, nmb, ntt, nxt);
                if (mb == kb) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int q = 0; q < 4; ++q) x[q] = mfma_f64(cur[q][u], acc[4 * kb + t][u], x[q]);
                    if (t == 3) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) acc[4 * kb + q] = x[q];
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc[4 * mb + q] = mfma_f64(cur[q][u], acc[4 * kb + t][u], acc[4 * mb + q]);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int u = 0; u < 4; ++u) cur[q][u] = nxt[q][u];
            }
        }
    }
    // The store's lane indices pass through an empty asm so that they are
    // formed here, not kept live (from the loads) across the whole solve.
    int gs = g, cs = c0 + r;
    asm volatile("" : "+v"(gs), "+v"(cs));
    if (cs < ncols) {
        double* bp = B + (int64_t)gs * ldb + cs;
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (16 * j + 4 * i + gs < n) bp[(int64_t)(16 * j + 4 * i) * ldb] = acc[j][i];
    }
}

inline unsigned nblk(int64_t n, int b = 256) {
    int64_t g = (n + b - 1) / b;
    return (unsigned)(g > 65535 * 16 ? 65535 * 16 : (g < 1 ? 1 : g));
}

}  // namespace

namespace ri {

int device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cached[dev] <= 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

hipError_t gemm_f64(bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
                    int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB,
                    double beta, double* C, int64_t ldc, int64_t sC, int batch, int tri,
                    int lowerC, hipStream_t s, int tile) {
    if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
    // 128-wide tiles when they still give a few hundred workgroups and K is
    // long enough to amortise the larger tile's staging (short K: 64-wide)
    const int64_t big_tiles = (int64_t)((M + 127) / 128) * ((N + 127) / 128) * batch;
    const bool big = tile ? tile == 128 : (M >= 128 && N >= 128 && big_tiles >= 200 && K > 128);
    if (big) {
        dim3 grid((N + 127) / 128, (M + 127) / 128, batch);
#define G128(a, b) gemm_f64_128_kernel<a, b><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, tri, lowerC)
        if (!ta && !tb) G128(false, false);
        else if (!ta && tb) G128(false, true);
        else if (ta && !tb) G128(true, false);
        else G128(true, true);
#undef G128
        return hipGetLastError();
    }
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch);
    if (!ta && !tb)
        gemm_f64_kernel<false, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, tri, lowerC);
    else if (!ta && tb)
        gemm_f64_kernel<false, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, tri, lowerC);
    else if (ta && !tb)
        gemm_f64_kernel<true, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, tri, lowerC);
    else
        gemm_f64_kernel<true, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, tri, lowerC);
    return hipGetLastError();
}

hipError_t cholesky_inv(double* A, int n, int64_t lda, double* Linv, int64_t ldi, double* dwork,
                        int* d_bad, hipStream_t s, const std::function<hipError_t(int)>& block_done) {
    const int nb = (n + 63) / 64;
    for (int k = 0; k < nb; ++k) {
        const int o = k * 64, w = min(64, n - o), rest = n - o - w;
        potrf_diag_kernel<<<1, 64, 0, s>>>(A, n, lda, k, dwork + (int64_t)k * 4096, d_bad);
        RI_TRY(hipGetLastError());
        if (rest > 0) {
            double* panel = A + (int64_t)(o + w) * lda + o;
            // panel <- panel * Dinv^T  (rows below the diagonal block)
            RI_TRY(gemm_f64(false, true, rest, w, w, 1.0, panel, lda, 0, dwork + (int64_t)k * 4096, 64, 0,
                            0.0, panel, lda, 0, 1, 0, 0, s));
        }
        if (block_done) RI_TRY(block_done(k));
        if (rest > 0) {
            double* panel = A + (int64_t)(o + w) * lda + o;
            // trailing lower update
            double* trail = A + (int64_t)(o + w) * lda + o + w;
            RI_TRY(gemm_f64(false, true, rest, rest, w, -1.0, panel, lda, 0, panel, lda, 0, 1.0, trail,
                            lda, 0, 1, 0, 1, s));
        }
    }
    zero_upper_kernel<<<nblk((int64_t)n * n), 256, 0, s>>>(A, n, lda);
    RI_TRY(hipGetLastError());
    if (!Linv) return hipSuccess;
    return tri_inverse(A, n, lda, dwork, Linv, ldi, s);
}

hipError_t tri_inverse_begin(double* Linv, int n, int64_t ldi, hipStream_t s) {
    identity_kernel<<<nblk((int64_t)n * n), 256, 0, s>>>(Linv, n, ldi);
    return hipGetLastError();
}

hipError_t tri_inverse_steps(const double* A, int n, int64_t lda, const double* dwork, double* Linv, int64_t ldi,
                             int k0, int k1, hipStream_t s) {
    // Solve L X = I by blocks: X_k = Dinv_k (I_k - L_{k,<k} X_{<k}).
    for (int k = k0; k < k1; ++k) {
        const int o = k * 64, w = min(64, n - o), rest = n - o - w, cols = o + w;
        double* Xk = Linv + (int64_t)o * ldi;
        RI_TRY(gemm_f64(false, false, w, cols, w, 1.0, dwork + (int64_t)k * 4096, 64, 0, Xk, ldi, 0, 0.0,
                        Xk, ldi, 0, 1, 0, 0, s));
        if (rest > 0)
            RI_TRY(gemm_f64(false, false, rest, cols, w, -1.0, A + (int64_t)(o + w) * lda + o, lda, 0, Xk,
                            ldi, 0, 1.0, Linv + (int64_t)(o + w) * ldi, ldi, 0, 1, 0, 0, s));
    }
    return hipSuccess;
}

hipError_t tri_inverse(const double* A, int n, int64_t lda, const double* dwork, double* Linv, int64_t ldi,
                       hipStream_t s) {
    RI_TRY(tri_inverse_begin(Linv, n, ldi, s));
    return tri_inverse_steps(A, n, lda, dwork, Linv, ldi, 0, (n + 63) / 64, s);
}

// Recursive form: B1 = L11^{-1} B1, B2 -= L21 B1, B2 = L22^{-1} B2, splitting
// at a multiple of 64 near the middle, so that half the flops run in one GEMM
// with K = n/2, a quarter in two with K = n/4, and so on; blocks of at most
// TRSM_LEAF rows are solved in one launch of the register-resident leaf
// kernel.  done(r0, r1) is called (in stream order) once rows r0 .. r1 of B
// are final.
constexpr int TRSM_LEAF = 256;
static_assert(TRSM_LEAF <= 256, "the leaf kernel holds at most four 64-row blocks");
hipError_t trsm_band(const double* L, int n, int64_t lda, const double* Dinv, double* P, hipStream_t s) {
    const int64_t total = (int64_t)((n + 63) / 64) * 4 * 4096;
    trsm_band_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(L, n, lda, Dinv, P);
    return hipGetLastError();
}

hipError_t trsm_rec(const double* L, int n, int64_t lda, const double* P, double* B, int ncols, int64_t ldb,
                    hipStream_t s, int r0, const std::function<hipError_t(int, int)>& done) {
    if (n <= 0) return hipSuccess;
    if (n <= TRSM_LEAF) {
        if (ncols > 0) {
            const unsigned grid = (unsigned)((ncols + 63) / 64);
            switch ((n + 63) / 64) {
                case 1: trsm_leaf_kernel<1><<<grid, 256, 0, s>>>(P, B, n, ncols, ldb); break;
                case 2: trsm_leaf_kernel<2><<<grid, 256, 0, s>>>(P, B, n, ncols, ldb); break;
                case 3: trsm_leaf_kernel<3><<<grid, 256, 0, s>>>(P, B, n, ncols, ldb); break;
                default: trsm_leaf_kernel<4><<<grid, 256, 0, s>>>(P, B, n, ncols, ldb); break;
            }
            RI_TRY(hipGetLastError());
        }
        return done ? done(r0, r0 + n) : hipSuccess;
    }
    const int n1 = max(64, n / 2 / 64 * 64), n2 = n - n1;
    RI_TRY(trsm_rec(L, n1, lda, P, B, ncols, ldb, s, r0, done));
    RI_TRY(gemm_f64(false, false, n2, ncols, n1, -1.0, L + (int64_t)n1 * lda, lda, 0, B, ldb, 0, 1.0,
                    B + (int64_t)n1 * ldb, ldb, 0, 1, 0, 0, s));
    return trsm_rec(L + (int64_t)n1 * lda + n1, n2, lda, P + (int64_t)(n1 / 64) * 4 * 4096, B + (int64_t)n1 * ldb,
                    ncols, ldb, s, r0 + n1, done);
}

hipError_t gemm_grouped(bool ta, bool tb, const GemmDesc* d, const int* prefix, int n, int total, hipStream_t s,
                        int tile) {
    if (total <= 0) return hipSuccess;
    if (tile == 128) {
        if (!ta && !tb) gemm_grouped128_kernel<false, false><<<total, 256, 0, s>>>(d, prefix, n);
        else if (!ta && tb) gemm_grouped128_kernel<false, true><<<total, 256, 0, s>>>(d, prefix, n);
        else if (ta && !tb) gemm_grouped128_kernel<true, false><<<total, 256, 0, s>>>(d, prefix, n);
        else gemm_grouped128_kernel<true, true><<<total, 256, 0, s>>>(d, prefix, n);
        return hipGetLastError();
    }
    if (tile != 64) return hipErrorInvalidValue;
    if (!ta && !tb) gemm_grouped_kernel<false, false><<<total, 256, 0, s>>>(d, prefix, n);
    else if (!ta && tb) gemm_grouped_kernel<false, true><<<total, 256, 0, s>>>(d, prefix, n);
    else if (ta && !tb) gemm_grouped_kernel<true, false><<<total, 256, 0, s>>>(d, prefix, n);
    else gemm_grouped_kernel<true, true><<<total, 256, 0, s>>>(d, prefix, n);
    return hipGetLastError();
}

hipError_t fill(double* p, double v, int64_t n, hipStream_t s) {
    fill_kernel<<<nblk(n), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    fill_i32_kernel<<<nblk(n), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}
hipError_t max_abs(const double* x, int64_t n, double* out, double* red, hipStream_t s) {
    maxabs_kernel<<<256, 1024, 0, s>>>(x, n, red);
    RI_TRY(hipGetLastError());
    maxabs_kernel<<<1, 1024, 0, s>>>(red, 256, out);
    return hipGetLastError();
}
hipError_t widen(const float* x, double* y, int64_t n, hipStream_t s) {
    f32_to_f64_kernel<<<nblk(n), 256, 0, s>>>(x, y, n);
    return hipGetLastError();
}
hipError_t copy(double* dst, const double* src, int64_t n, hipStream_t s) {
    return hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s);
}

}  // namespace ri
