// RI Fock build: decompression of the fitted tensor into packed symmetric
// tiles, the exchange half-transform X^P = B^P C_occ on MFMA, the exchange
// SYRK K = sum_P X^P X^P^T over lower tiles with split-K, and the
// bandwidth-bound Coulomb contractions gamma = B:D, J = sum_P gamma_P B^P on
// the compressed (significant-pair) tensor.
#include "kernels.h"

namespace {

__device__ __forceinline__ void tile_ij(int t, int& I, int& J) {
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
}

__global__ void pair_map_kernel(const int32_t* pairs, int64_t n_pairs, int N, int32_t* map) {
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    map[(int64_t)pairs[2 * q] * N + pairs[2 * q + 1]] = (int32_t)q;
}

// B[P][tile][r*64+c] = Bc[P][pair(64I+r, 64J+c)] or 0.
template <typename T>
__global__ __launch_bounds__(256) void pack_kernel(const double* Bc, int64_t n_pairs, const int32_t* map,
                                                   int N, int64_t ntl, T* B) {
    const int t = blockIdx.x, P = blockIdx.y;
    int I, J;
    tile_ij(t, I, J);
    const double* row = Bc + (int64_t)P * n_pairs;
    T* out = B + ((int64_t)P * ntl + t) * 4096;
    for (int e = threadIdx.x; e < 4096; e += 256) {
        int mu = 64 * I + (e >> 6), nu = 64 * J + (e & 63);
        double v = 0.0;
        if (mu < N && nu < N) {
            int m = max(mu, nu), n = min(mu, nu);
            int32_t q = map[(int64_t)m * N + n];
            if (q >= 0) v = row[q];
        }
        out[e] = (T)v;
    }
}

// X^T for one (row-block I, auxiliary P): Xt[P][i][64I + m] = sum_nu C[nu][i] B^P[64I+m][nu].
// MFMA rows = occupied index i (MT tiles of 16), columns = mu (4 waves x 16).
template <int MT>
__global__ __launch_bounds__(256) void x_kernel_f64(const double* __restrict__ B, int nt, int64_t ntl,
                                                    const double* __restrict__ C, int N, int n_occ,
                                                    double* __restrict__ Xt, int Npad) {
    const int I = blockIdx.x, P = blockIdx.y, i0 = blockIdx.z * 128;
    const double* Bp = B + (int64_t)P * ntl * 4096;
    constexpr int W = MT * 16;
    __shared__ double Cs[16][W + 1];
    __shared__ double Bs[16][65];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
    d4_t acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = d4_t{0.0, 0.0, 0.0, 0.0};
    for (int J = 0; J < nt; ++J) {
        const bool lower = J <= I;
        const double* tp = Bp + (int64_t)(lower ? (I * (I + 1) / 2 + J) : (J * (J + 1) / 2 + I)) * 4096;
        for (int k0 = 0; k0 < 64; k0 += 16) {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (lower) {
                    int k = tid & 15, m = (tid >> 4) + 16 * r;
                    Bs[k][m] = tp[m * 64 + k0 + k];
                } else {
                    int m = tid & 63, k = (tid >> 6) + 4 * r;
                    Bs[k][m] = tp[(k0 + k) * 64 + m];
                }
            }
            for (int e = tid; e < 16 * W; e += 256) {
                int k = e / W, i = e % W;
                int nu = 64 * J + k0 + k, gi = i0 + i;
                Cs[k][i] = (nu < N && gi < n_occ) ? C[(int64_t)nu * n_occ + gi] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                double b = Bs[kk + lk][wave * 16 + li];
#pragma unroll
                for (int m = 0; m < MT; ++m) acc[m] = mfma_f64(Cs[kk + lk][m * 16 + li], b, acc[m]);
            }
        }
    }
    const int mu = 64 * I + wave * 16 + li;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int i = i0 + m * 16 + 4 * r + lk;
            if (i < n_occ) Xt[((int64_t)P * n_occ + i) * Npad + mu] = acc[m][r];
        }
}

__global__ void kreduce_kernel(const double* part, int n_split, int Npad, int N, double* K) {
    int nu = blockIdx.x * blockDim.x + threadIdx.x, mu = blockIdx.y;
    if (nu > mu || mu >= N) return;
    double s = 0.0;
    for (int k = 0; k < n_split; ++k) s += part[((int64_t)k * Npad + mu) * Npad + nu];
    K[(int64_t)mu * N + nu] = s;
    K[(int64_t)nu * N + mu] = s;
}

// dpair[q] = w_q D_mu_nu,  D = 2 C C^T,  w = 1 on the diagonal, 2 off it.
__global__ void dpair_kernel(const int32_t* pairs, int64_t n_pairs, const double* C, int n_occ,
                             double* dp) {
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    int mu = pairs[2 * q], nu = pairs[2 * q + 1];
    const double* a = C + (int64_t)mu * n_occ;
    const double* b = C + (int64_t)nu * n_occ;
    double s = 0.0;
    for (int i = 0; i < n_occ; ++i) s += a[i] * b[i];
    dp[q] = (mu == nu ? 2.0 : 4.0) * s;
}

__global__ __launch_bounds__(256) void gamma_kernel(const double* Bc, int64_t n_pairs, const double* dp,
                                                    double* gamma) {
    const int P = blockIdx.x;
    const double* row = Bc + (int64_t)P * n_pairs;
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < n_pairs; q += 256) s += row[q] * dp[q];
    __shared__ double sh[4];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) gamma[P] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void jpair_kernel(const double* Bc, int64_t n_pairs, int n_aux, const double* gamma,
                             int per, double* jpart) {
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    int p0 = blockIdx.y * per, p1 = min(n_aux, p0 + per);
    double s = 0.0;
    for (int P = p0; P < p1; ++P) s += Bc[(int64_t)P * n_pairs + q] * gamma[P];
    jpart[(int64_t)blockIdx.y * n_pairs + q] = s;
}

__global__ void jscatter_kernel(const double* jpart, int n_split, const int32_t* pairs,
                                int64_t n_pairs, int N, double* J) {
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    double s = 0.0;
    for (int k = 0; k < n_split; ++k) s += jpart[(int64_t)k * n_pairs + q];
    int mu = pairs[2 * q], nu = pairs[2 * q + 1];
    J[(int64_t)mu * N + nu] = s;
    J[(int64_t)nu * N + mu] = s;
}

}  // namespace

namespace ri {

hipError_t pair_map(const int32_t* pairs, int64_t n_pairs, int N, int32_t* map, hipStream_t st) {
    RI_TRY(fill_i32(map, -1, (int64_t)N * N, st));
    if (n_pairs == 0) return hipSuccess;
    pair_map_kernel<<<(unsigned)((n_pairs + 255) / 256), 256, 0, st>>>(pairs, n_pairs, N, map);
    return hipGetLastError();
}

hipError_t pack_b(const double* Bc, int64_t n_pairs, const int32_t* map, int N, int n_aux, void* B,
                  int prec, hipStream_t st) {
    dim3 grid((unsigned)n_tiles(N), n_aux);
    if (prec == RI_FP64)
        pack_kernel<double><<<grid, 256, 0, st>>>(Bc, n_pairs, map, N, n_tiles(N), (double*)B);
    else if (prec == RI_FP32)
        pack_kernel<float><<<grid, 256, 0, st>>>(Bc, n_pairs, map, N, n_tiles(N), (float*)B);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t x_transform(const void* B, int prec, int N, int n_aux, int n_occ, const double* C, void* Xt,
                       hipStream_t st) {
    const int nt = n_tiles_1d(N), Npad = nt * 64;
    if (prec != RI_FP64) return hipErrorInvalidValue;
    const int mt = (min(n_occ, 128) + 15) / 16;
    dim3 grid(nt, n_aux, (n_occ + 127) / 128);
    const double* b = (const double*)B;
    double* x = (double*)Xt;
    const int64_t ntl = n_tiles(N);
    switch (mt) {
#define XCASE(k) case k: x_kernel_f64<k><<<grid, 256, 0, st>>>(b, nt, ntl, C, N, n_occ, x, Npad); break;
        XCASE(1) XCASE(2) XCASE(3) XCASE(4) XCASE(5) XCASE(6) XCASE(7) XCASE(8)
#undef XCASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int k_split_count(int N, int n_aux, int n_occ) {
    const int nt = n_tiles_1d(N);
    const int64_t tiles = (int64_t)nt * (nt + 1) / 2;
    int64_t rows = (int64_t)n_aux * n_occ;
    int s = (int)((2048 + tiles - 1) / tiles);
    if (s < 1) s = 1;
    if (s > 64) s = 64;
    if (rows < (int64_t)s * 64) s = (int)((rows + 63) / 64);
    return s < 1 ? 1 : s;
}

hipError_t k_syrk(const void* Xt, int prec, int N, int n_aux, int n_occ, double* part, int n_split,
                  double* K, hipStream_t st) {
    if (prec != RI_FP64) return hipErrorInvalidValue;
    const int nt = n_tiles_1d(N), Npad = nt * 64;
    const int64_t rows = (int64_t)n_aux * n_occ;
    const int64_t chunk = ((rows + n_split - 1) / n_split + 15) / 16 * 16;
    const double* x = (const double*)Xt;
    const int64_t sq = (int64_t)Npad * Npad;
    int full = (int)(rows / chunk);
    if (full > n_split) full = n_split;
    if (full > 0)
        RI_TRY(gemm_f64(true, false, Npad, Npad, (int)chunk, 1.0, x, Npad, chunk * Npad, x, Npad,
                        chunk * Npad, 0.0, part, Npad, sq, full, 0, 1, st));
    int used = full;
    int64_t rem = rows - (int64_t)full * chunk;
    if (rem > 0) {
        const double* xr = x + (int64_t)full * chunk * Npad;
        RI_TRY(gemm_f64(true, false, Npad, Npad, (int)rem, 1.0, xr, Npad, 0, xr, Npad, 0, 0.0,
                        part + (int64_t)full * sq, Npad, 0, 1, 0, 1, st));
        ++used;
    }
    dim3 grid((N + 255) / 256, N);
    kreduce_kernel<<<grid, 256, 0, st>>>(part, used, Npad, N, K);
    return hipGetLastError();
}

int j_split_count(int n_aux) { return n_aux >= 512 ? 16 : 1; }

hipError_t gamma_j(const double* Bc, const int32_t* pairs, int64_t n_pairs, int N, int n_aux, int n_occ,
                   const double* C, double* dpair, double* gamma, double* jpart, int n_jsplit, double* J,
                   hipStream_t st) {
    RI_TRY(fill(J, 0.0, (int64_t)N * N, st));
    if (n_pairs == 0) return fill(gamma, 0.0, n_aux, st);
    const unsigned pb = (unsigned)((n_pairs + 255) / 256);
    dpair_kernel<<<pb, 256, 0, st>>>(pairs, n_pairs, C, n_occ, dpair);
    RI_TRY(hipGetLastError());
    gamma_kernel<<<n_aux, 256, 0, st>>>(Bc, n_pairs, dpair, gamma);
    RI_TRY(hipGetLastError());
    const int per = (n_aux + n_jsplit - 1) / n_jsplit;
    jpair_kernel<<<dim3(pb, n_jsplit), 256, 0, st>>>(Bc, n_pairs, n_aux, gamma, per, jpart);
    RI_TRY(hipGetLastError());
    jscatter_kernel<<<pb, 256, 0, st>>>(jpart, n_jsplit, pairs, n_pairs, N, J);
    return hipGetLastError();
}

}  // namespace ri
