// Learned SCF start (project extension): per-pair features, a 3-layer MLP
// (width 256, SiLU) trained in FP32 with its own forward, backward and Adam
// kernels, BF16 inference for the 256 x 256 layer, and the scatter of
// predicted pair densities into a dense symmetric matrix.
#include "kernels.h"

#include <algorithm>

namespace {

constexpr int NF = RI_MLP_NFEAT;
constexpr int W = RI_MLP_WIDTH;

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}
__device__ __forceinline__ f4_t mfma_f32x4(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// f0 |A-B|, f1 ln max(a,b), f2 ln min(a,b), f3 same centre, f4 exp(-(ab/(a+b))|A-B|^2),
// f5/f6 max/min coordination sum_{C != X} exp(-|R_X - R_C|^2 / 8),
// f7 sum_C exp(-|P - R_C|^2 / 4) at the Gaussian product centre P.
__global__ void features_kernel(const double* xyz, int nc, const int32_t* fc, const double* fe,
                                const int32_t* pairs, int64_t n_pairs, float* feat) {
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    int mu = pairs[2 * q], nu = pairs[2 * q + 1];
    int ca = fc[mu], cb = fc[nu];
    double a = fe[mu], b = fe[nu];
    const double* A = xyz + 3 * ca;
    const double* B = xyz + 3 * cb;
    double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
    double r2 = dx * dx + dy * dy + dz * dz;
    double Px = (a * A[0] + b * B[0]) / (a + b), Py = (a * A[1] + b * B[1]) / (a + b),
           Pz = (a * A[2] + b * B[2]) / (a + b);
    double cA = 0.0, cB = 0.0, md = 0.0;
    for (int c = 0; c < nc; ++c) {
        const double* C = xyz + 3 * c;
        double ax = A[0] - C[0], ay = A[1] - C[1], az = A[2] - C[2];
        double bx = B[0] - C[0], by = B[1] - C[1], bz = B[2] - C[2];
        double px = Px - C[0], py = Py - C[1], pz = Pz - C[2];
        if (c != ca) cA += exp(-(ax * ax + ay * ay + az * az) / 8.0);
        if (c != cb) cB += exp(-(bx * bx + by * by + bz * bz) / 8.0);
        md += exp(-(px * px + py * py + pz * pz) / 4.0);
    }
    float* f = feat + q * NF;
    f[0] = (float)sqrt(r2);
    f[1] = (float)log(fmax(a, b));
    f[2] = (float)log(fmin(a, b));
    f[3] = ca == cb ? 1.0f : 0.0f;
    f[4] = (float)exp(-(a * b / (a + b)) * r2);
    f[5] = (float)fmax(cA, cB);
    f[6] = (float)fmin(cA, cB);
    f[7] = (float)md;
}

// layer 1: z1 = ((f - mu) / sigma) W1 + b1 (keeps x-hat for the backward), h1 = silu(z1)
__global__ void layer1_kernel(const float* feat, int64_t n, const float* mu, const float* sg, const float* W1,
                              const float* b1, float* xh, float* z1, float* h1) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * W) return;
    int64_t r = e / W;
    int c = e % W;
    float s = b1[c];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        float x = (feat[r * NF + k] - mu[k]) / sg[k];
        s += x * W1[k * W + c];
        if (c == 0) xh[r * NF + k] = x;
    }
    z1[e] = s;
    h1[e] = silu(s);
}

// C[M][N] = op(A) op(B) (+ bias[N]) with optional silu epilogue, FP32 MFMA,
// 64 x 64 tiles staged through LDS.  A: TA ? [K][M] : [M][K]; B: TB ? [N][K] : [K][N].
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f32_kernel(int M, int N, int K, const float* __restrict__ A,
                                                       int lda, const float* __restrict__ B, int ldb,
                                                       float* __restrict__ C, int ldc, const float* bias,
                                                       float* Cact) {
    __shared__ float As[16][65];
    __shared__ float Bs[16][65];
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < K; k0 += 16) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int m, k;
            if (!TA) { k = tid & 15; m = (tid >> 4) + 16 * r; }
            else     { m = tid & 63; k = (tid >> 6) + 4 * r; }
            int gm = m0 + m, gk = k0 + k;
            As[k][m] = (gm < M && gk < K) ? (TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk]) : 0.0f;
            int n, kb;
            if (!TB) { n = tid & 63; kb = (tid >> 6) + 4 * r; }
            else     { kb = tid & 15; n = (tid >> 4) + 16 * r; }
            int gn = n0 + n, gkb = k0 + kb;
            Bs[kb][n] = (gn < N && gkb < K) ? (TB ? B[(int64_t)gn * ldb + gkb] : B[(int64_t)gkb * ldb + gn]) : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            float a0 = As[kk + lk][wm + li], a1 = As[kk + lk][wm + 16 + li];
            float b0 = Bs[kk + lk][wn + li], b1 = Bs[kk + lk][wn + 16 + li];
            acc[0][0] = mfma_f32x4(a0, b0, acc[0][0]);
            acc[0][1] = mfma_f32x4(a0, b1, acc[0][1]);
            acc[1][0] = mfma_f32x4(a1, b0, acc[1][0]);
            acc[1][1] = mfma_f32x4(a1, b1, acc[1][1]);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int gm = m0 + wm + 16 * i + 4 * lk + r, gn = n0 + wn + 16 * j + li;
                if (gm < M && gn < N) {
                    float v = acc[i][j][r] + (bias ? bias[gn] : 0.0f);
                    C[(int64_t)gm * ldc + gn] = v;
                    if (Cact) Cact[(int64_t)gm * ldc + gn] = silu(v);
                }
            }
}

// z2 = h1 W2 + b2 with BF16 operands (h1 and W2^T converted on the fly) and
// FP32 accumulation: v_mfma_f32_16x16x32_bf16, lane l supplies rows l%16 and
// k = 8 (l/16) + 0..7, receives D[4 (l/16) + r][l%16].  One wave per 16 x 64
// output block, operands read directly from global memory.
__global__ __launch_bounds__(256) void layer2_bf16_kernel(const float* __restrict__ h1, int64_t n,
                                                          const __bf16* __restrict__ W2t, const float* b2,
                                                          float* __restrict__ z2, float* __restrict__ h2) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int64_t r0 = (blockIdx.x * 4 + wave) * 16;
    const int c0 = blockIdx.y * 64;
    if (r0 >= n) return;
    f4_t acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f4_t{0, 0, 0, 0};
    const int64_t row = min(r0 + li, n - 1);
    for (int k0 = 0; k0 < W; k0 += 32) {
        bf16x8_t a;
        const float* hp = h1 + row * W + k0 + 8 * lk;
#pragma unroll
        for (int t = 0; t < 8; ++t) a[t] = (__bf16)hp[t];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bf16x8_t b = *(const bf16x8_t*)(W2t + (int64_t)(c0 + 16 * j + li) * W + k0 + 8 * lk);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int64_t gr = r0 + 4 * lk + r;
            int gc = c0 + 16 * j + li;
            if (gr < n) {
                float v = acc[j][r] + b2[gc];
                z2[gr * W + gc] = v;
                h2[gr * W + gc] = silu(v);
            }
        }
}

__global__ void transpose_bf16_kernel(const float* W2, __bf16* W2t) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= W * W) return;
    int k = e / W, c = e % W;
    W2t[c * W + k] = (__bf16)W2[e];
}

// y = h2 w3 + b3: one wave per row
__global__ __launch_bounds__(256) void layer3_kernel(const float* h2, int64_t n, const float* w3, const float* b3,
                                                     float* y) {
    const int lane = threadIdx.x & 63;
    const int64_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    float s = 0.0f;
    for (int c = lane; c < W; c += 64) s += h2[r * W + c] * w3[c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if (lane == 0) y[r] = s + b3[0];
}

// dy = 2 (y - t) / n, partial sums of (y - t)^2 per block
__global__ __launch_bounds__(256) void mse_kernel(const float* y, const float* t, int64_t n, float* dy,
                                                  float* part) {
    int64_t i = blockIdx.x * 256ll + threadIdx.x;
    float r = 0.0f;
    if (i < n) {
        r = y[i] - t[i];
        dy[i] = 2.0f * r / (float)n;
    }
    float s = r * r;
    __shared__ float sh[4];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void sum_kernel(const float* part, int np, float scale, float* out) {
    if (threadIdx.x != 0) return;
    float s = 0.0f;
    for (int i = 0; i < np; ++i) s += part[i];
    *out = s * scale;
}

// dz2 = dy (x) w3 * silu'(z2), in place over z2's buffer
__global__ void dz2_kernel(const float* dy, const float* w3, int64_t n, float* z2) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * W) return;
    z2[e] = dy[e / W] * w3[e % W] * dsilu(z2[e]);
}

// dz1 = dh1 * silu'(z1), in place over dh1
__global__ void dz1_kernel(const float* z1, int64_t n, float* dh1) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * W) return;
    dh1[e] *= dsilu(z1[e]);
}

// column sums of A [n][cols] over row chunks: part[blk][c]
__global__ void colsum_partial_kernel(const float* A, int64_t n, int cols, int64_t rows_per, float* part) {
    int c = threadIdx.x + blockIdx.y * blockDim.x;
    if (c >= cols) return;
    int64_t r0 = blockIdx.x * rows_per, r1 = min(n, r0 + rows_per);
    float s = 0.0f;
    for (int64_t r = r0; r < r1; ++r) s += A[r * cols + c];
    part[(int64_t)blockIdx.x * cols + c] = s;
}
__global__ void colsum_final_kernel(const float* part, int nblk, int cols, float* out) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * cols + c];
    out[c] = s;
}

// g_w3[c] = sum_r h2[r][c] dy[r] (partials over row chunks)
__global__ void gw3_partial_kernel(const float* h2, const float* dy, int64_t n, int64_t rows_per, float* part) {
    int c = threadIdx.x;
    int64_t r0 = blockIdx.x * rows_per, r1 = min(n, r0 + rows_per);
    float s = 0.0f;
    for (int64_t r = r0; r < r1; ++r) s += h2[r * W + c] * dy[r];
    part[(int64_t)blockIdx.x * W + c] = s;
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void scatter_density_kernel(const int32_t* pairs, int64_t n_pairs, const float* d, int N, double* D) {
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    int mu = pairs[2 * q], nu = pairs[2 * q + 1];
    double v = d[q];
    D[(int64_t)mu * N + nu] = v;
    D[(int64_t)nu * N + mu] = v;
}

__global__ void gather_density_kernel(const int32_t* pairs, int64_t n_pairs, const double* D, int N, float* d) {
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    d[q] = (float)D[(int64_t)pairs[2 * q] * N + pairs[2 * q + 1]];
}

// Distance^2 of the pair's centres, the coordination sum c_A + c_B and the
// Gaussian-product-centre density (f7 above) of one geometry.
__device__ __forceinline__ void pair_geometry(const double* xyz, int nc, int ca, int cb, double a, double b,
                                              double& r2, double& csum, double& md) {
    const double* A = xyz + 3 * ca;
    const double* B = xyz + 3 * cb;
    const double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
    r2 = dx * dx + dy * dy + dz * dz;
    const double Px = (a * A[0] + b * B[0]) / (a + b), Py = (a * A[1] + b * B[1]) / (a + b),
                 Pz = (a * A[2] + b * B[2]) / (a + b);
    double cA = 0.0, cB = 0.0, m = 0.0;
    for (int c = 0; c < nc; ++c) {
        const double* C = xyz + 3 * c;
        const double ax = A[0] - C[0], ay = A[1] - C[1], az = A[2] - C[2];
        const double bx = B[0] - C[0], by = B[1] - C[1], bz = B[2] - C[2];
        const double px = Px - C[0], py = Py - C[1], pz = Pz - C[2];
        if (c != ca) cA += exp(-(ax * ax + ay * ay + az * az) / 8.0);
        if (c != cb) cB += exp(-(bx * bx + by * by + bz * bz) / 8.0);
        m += exp(-(px * px + py * py + pz * pz) / 4.0);
    }
    csum = cA + cB;
    md = m;
}

// Features of a pair for the density change between the previous geometry
// (xyz0, converged density Dp) and the new one (xyz): g0 = Dp[mu][nu],
// g1 = change of |A - B|, g2 = change of exp(-(ab/(a+b))|A-B|^2), g3/g4 =
// ln max/min(a, b), g5 = same centre, g6 = change of c_A + c_B, g7 = change of
// the product-centre density.
__global__ void delta_features_kernel(const double* xyz, const double* xyz0, int nc, const int32_t* fc,
                                      const double* fe, const int32_t* pairs, int64_t n_pairs, const double* Dp,
                                      int N, float* feat) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    const int mu = pairs[2 * q], nu = pairs[2 * q + 1];
    const int ca = fc[mu], cb = fc[nu];
    const double a = fe[mu], b = fe[nu], e = a * b / (a + b);
    double r2, cs, md, r20, cs0, md0;
    pair_geometry(xyz, nc, ca, cb, a, b, r2, cs, md);
    pair_geometry(xyz0, nc, ca, cb, a, b, r20, cs0, md0);
    float* f = feat + q * NF;
    f[0] = (float)Dp[(int64_t)mu * N + nu];
    f[1] = (float)(sqrt(r2) - sqrt(r20));
    f[2] = (float)(exp(-e * r2) - exp(-e * r20));
    f[3] = (float)log(fmax(a, b));
    f[4] = (float)log(fmin(a, b));
    f[5] = ca == cb ? 1.0f : 0.0f;
    f[6] = (float)(cs - cs0);
    f[7] = (float)(md - md0);
}

// d[q] = scale (Dn - Dp)[mu][nu] on the listed pairs
__global__ void density_change_kernel(const int32_t* pairs, int64_t n_pairs, const double* Dn, const double* Dp,
                                      int N, float scale, float* d) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    const int64_t i = (int64_t)pairs[2 * q] * N + pairs[2 * q + 1];
    d[q] = (float)((double)scale * (Dn[i] - Dp[i]));
}

// Dout[mu][nu] = Dout[nu][mu] = Dp[mu][nu] + scale d[q] on the listed pairs
// (Dout holds a copy of Dp elsewhere)
__global__ void density_add_kernel(const int32_t* pairs, int64_t n_pairs, const float* d, double scale,
                                   const double* Dp, int N, double* Dout) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    const int mu = pairs[2 * q], nu = pairs[2 * q + 1];
    const double v = Dp[(int64_t)mu * N + nu] + scale * (double)d[q];
    Dout[(int64_t)mu * N + nu] = v;
    Dout[(int64_t)nu * N + mu] = v;
}

inline unsigned g1(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

template <bool TA, bool TB>
hipError_t gemm_f32(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
                    const float* bias, float* Cact, hipStream_t st) {
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    gemm_f32_kernel<TA, TB><<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc, bias, Cact);
    return hipGetLastError();
}

}  // namespace

namespace ri {

hipError_t pair_features(const ri_system* s, const int32_t* pairs, int64_t n_pairs, float* feat, hipStream_t st) {
    if (n_pairs == 0) return hipSuccess;
    features_kernel<<<g1(n_pairs), 256, 0, st>>>(s->xyz, s->n_centres, s->fn_centre, s->fn_exp, pairs, n_pairs, feat);
    return hipGetLastError();
}

MlpWS carve_mlp(char* base, size_t cap, size_t& off, int64_t n) {
    auto take = [&](int64_t cnt, size_t esz) {
        size_t b = ((size_t)cnt * esz + 255) & ~(size_t)255;
        size_t o = off;
        off += b;
        return base ? (void*)(base + o) : nullptr;
    };
    MlpWS w;
    w.xh = (float*)take(n * NF, 4);
    w.z1 = (float*)take(n * W, 4);
    w.h1 = (float*)take(n * W, 4);
    w.z2 = (float*)take(n * W, 4);
    w.h2 = (float*)take(n * W, 4);
    w.y = (float*)take(n, 4);
    w.dy = (float*)take(n, 4);
    w.part = (float*)take((int64_t)std::max<int64_t>(1024, (n + 255) / 256) * W, 4);
    w.grad = (float*)take(RI_MLP_NPARAM, 4);
    w.W2t = (__bf16*)take(W * W, 2);
    (void)cap;
    return w;
}

hipError_t mlp_forward(const ri_mlp* net, const float* feat, int64_t n, float* y, int prec, const MlpWS& w,
                       hipStream_t st) {
    const float* P = net->params;
    layer1_kernel<<<g1(n * W), 256, 0, st>>>(feat, n, net->mu, net->sigma, P + RI_MLP_OFF_W1, P + RI_MLP_OFF_B1,
                                             w.xh, w.z1, w.h1);
    RI_TRY(hipGetLastError());
    if (prec == RI_MLP_BF16) {
        transpose_bf16_kernel<<<g1(W * W), 256, 0, st>>>(P + RI_MLP_OFF_W2, w.W2t);
        RI_TRY(hipGetLastError());
        dim3 grid((unsigned)((n + 63) / 64), W / 64);
        layer2_bf16_kernel<<<grid, 256, 0, st>>>(w.h1, n, w.W2t, P + RI_MLP_OFF_B2, w.z2, w.h2);
    } else {
        RI_TRY((gemm_f32<false, false>((int)n, W, W, w.h1, W, P + RI_MLP_OFF_W2, W, w.z2, W, P + RI_MLP_OFF_B2, w.h2, st)));
    }
    RI_TRY(hipGetLastError());
    layer3_kernel<<<g1(n, 4), 256, 0, st>>>(w.h2, n, P + RI_MLP_OFF_W3, P + RI_MLP_OFF_B3, y);
    return hipGetLastError();
}

hipError_t mlp_train_step(const ri_mlp* net, float* m, float* v, int step, float lr, const float* feat,
                          const float* target, int64_t n, float* loss, const MlpWS& w, hipStream_t st) {
    float* P = net->params;
    RI_TRY(mlp_forward(net, feat, n, w.y, RI_MLP_FP32, w, st));
    const int nb = (int)g1(n);
    mse_kernel<<<nb, 256, 0, st>>>(w.y, target, n, w.dy, w.part);
    RI_TRY(hipGetLastError());
    sum_kernel<<<1, 64, 0, st>>>(w.part, nb, 1.0f / (float)n, loss);
    RI_TRY(hipGetLastError());
    float* g = w.grad;
    const int64_t rows_per = 256;
    const int nchunk = (int)((n + rows_per - 1) / rows_per);
    // w3, b3
    gw3_partial_kernel<<<nchunk, W, 0, st>>>(w.h2, w.dy, n, rows_per, w.part);
    colsum_final_kernel<<<1, W, 0, st>>>(w.part, nchunk, W, g + RI_MLP_OFF_W3);
    colsum_partial_kernel<<<dim3(nchunk, 1), 1, 0, st>>>(w.dy, n, 1, rows_per, w.part);
    colsum_final_kernel<<<1, 1, 0, st>>>(w.part, nchunk, 1, g + RI_MLP_OFF_B3);
    RI_TRY(hipGetLastError());
    // dz2 (in z2's buffer)
    dz2_kernel<<<g1(n * W), 256, 0, st>>>(w.dy, P + RI_MLP_OFF_W3, n, w.z2);
    RI_TRY(hipGetLastError());
    // g_W2 = h1^T dz2, g_b2 = colsum dz2
    RI_TRY((gemm_f32<true, false>(W, W, (int)n, w.h1, W, w.z2, W, g + RI_MLP_OFF_W2, W, nullptr, nullptr, st)));
    colsum_partial_kernel<<<dim3(nchunk, 1), W, 0, st>>>(w.z2, n, W, rows_per, w.part);
    colsum_final_kernel<<<1, W, 0, st>>>(w.part, nchunk, W, g + RI_MLP_OFF_B2);
    RI_TRY(hipGetLastError());
    // dh1 = dz2 W2^T (into h2's buffer), dz1 = dh1 silu'(z1)
    RI_TRY((gemm_f32<false, true>((int)n, W, W, w.z2, W, P + RI_MLP_OFF_W2, W, w.h2, W, nullptr, nullptr, st)));
    dz1_kernel<<<g1(n * W), 256, 0, st>>>(w.z1, n, w.h2);
    RI_TRY(hipGetLastError());
    // g_W1 = xh^T dz1, g_b1 = colsum dz1
    RI_TRY((gemm_f32<true, false>(NF, W, (int)n, w.xh, NF, w.h2, W, g + RI_MLP_OFF_W1, W, nullptr, nullptr, st)));
    colsum_partial_kernel<<<dim3(nchunk, 1), W, 0, st>>>(w.h2, n, W, rows_per, w.part);
    colsum_final_kernel<<<1, W, 0, st>>>(w.part, nchunk, W, g + RI_MLP_OFF_B1);
    RI_TRY(hipGetLastError());
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    adam_kernel<<<g1(RI_MLP_NPARAM), 256, 0, st>>>(P, g, m, v, RI_MLP_NPARAM, lr, b1, b2, 1e-8f, c1, c2);
    return hipGetLastError();
}

hipError_t scatter_density(int N, const int32_t* pairs, int64_t n_pairs, const float* d, double* D, hipStream_t st) {
    RI_TRY(fill(D, 0.0, (int64_t)N * N, st));
    if (n_pairs == 0) return hipSuccess;
    scatter_density_kernel<<<g1(n_pairs), 256, 0, st>>>(pairs, n_pairs, d, N, D);
    return hipGetLastError();
}

hipError_t pair_delta_features(const ri_system* s, const double* xyz_prev, const int32_t* pairs, int64_t n_pairs,
                               const double* D_prev, float* feat, hipStream_t st) {
    if (n_pairs == 0) return hipSuccess;
    delta_features_kernel<<<g1(n_pairs), 256, 0, st>>>(s->xyz, xyz_prev, s->n_centres, s->fn_centre, s->fn_exp,
                                                        pairs, n_pairs, D_prev, s->n_fn, feat);
    return hipGetLastError();
}

hipError_t density_change(int N, const int32_t* pairs, int64_t n_pairs, const double* Dn, const double* Dp,
                          float scale, float* d, hipStream_t st) {
    if (n_pairs == 0) return hipSuccess;
    density_change_kernel<<<g1(n_pairs), 256, 0, st>>>(pairs, n_pairs, Dn, Dp, N, scale, d);
    return hipGetLastError();
}

hipError_t density_add(int N, const int32_t* pairs, int64_t n_pairs, const float* d, double scale, const double* Dp,
                       double* Dout, hipStream_t st) {
    RI_TRY(copy(Dout, Dp, (int64_t)N * N, st));
    if (n_pairs == 0) return hipSuccess;
    density_add_kernel<<<g1(n_pairs), 256, 0, st>>>(pairs, n_pairs, d, scale, Dp, N, Dout);
    return hipGetLastError();
}

hipError_t gather_density(int N, const int32_t* pairs, int64_t n_pairs, const double* D, float* d, hipStream_t st) {
    if (n_pairs == 0) return hipSuccess;
    gather_density_kernel<<<g1(n_pairs), 256, 0, st>>>(pairs, n_pairs, D, N, d);
    return hipGetLastError();
}

}  // namespace ri
