// Exchange from a density matrix alone (no occupied orbitals), as needed by
// a density start of the SCF: K = 1/2 sum_P B^P D B^P, the RI form of the
// exchange operator for any D.  Slabs of S auxiliaries at a time: full square
// B^P unpacked from B_c, one batched GEMM Y^P = B^P D into a side-by-side
// panel Y = [Y^1 .. Y^S], and one GEMM K += 1/2 Y [B^1; ..; B^S] whose inner
// dimension runs over (P, sigma).
#include "kernels.h"

#include <algorithm>

namespace {

// Bf[p][mu][nu] = B_c[p][pair(max, min)] or 0
__global__ void unpack_full_kernel(const double* __restrict__ Bc, int64_t n_pairs, const int32_t* __restrict__ map,
                                   int N, double* __restrict__ Bf) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t n2 = (int64_t)N * N;
    if (e >= n2) return;
    const int p = blockIdx.y;
    const int mu = (int)(e / N), nu = (int)(e % N);
    const int32_t q = map[(int64_t)max(mu, nu) * N + min(mu, nu)];
    Bf[p * n2 + e] = q >= 0 ? Bc[(int64_t)p * n_pairs + q] : 0.0;
}

// K <- (K + K^T) / 2
__global__ void symmetrize_kernel(double* K, int N) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    const int i = (int)(e / N), j = (int)(e % N);
    if (j >= i) return;
    const double v = 0.5 * (K[(int64_t)i * N + j] + K[(int64_t)j * N + i]);
    K[(int64_t)i * N + j] = v;
    K[(int64_t)j * N + i] = v;
}

}  // namespace

namespace ri {

hipError_t k_density(const double* Bc, const int32_t* pairs, int64_t n_pairs, int N, int n_aux, const double* D,
                     int32_t* map, double* Bf, double* Y, int S, double* K, hipStream_t st) {
    const int64_t n2 = (int64_t)N * N;
    if (n_pairs == 0) return fill(K, 0.0, n2, st);
    RI_TRY(pair_map(pairs, n_pairs, N, map, st));
    for (int P0 = 0; P0 < n_aux; P0 += S) {
        const int s = std::min(S, n_aux - P0);
        unpack_full_kernel<<<dim3((unsigned)((n2 + 255) / 256), s), 256, 0, st>>>(Bc + (int64_t)P0 * n_pairs, n_pairs,
                                                                                  map, N, Bf);
        RI_TRY(hipGetLastError());
        // Y[:, p N + sigma] = (B^p D)[:, sigma]
        RI_TRY(gemm_f64(false, false, N, N, N, 1.0, Bf, N, n2, D, N, 0, 0.0, Y, (int64_t)S * N, N, s, 0, 0, st));
        // K (+)= 1/2 Y [B^1; ..; B^s]
        RI_TRY(gemm_f64(false, false, N, N, s * N, 0.5, Y, (int64_t)S * N, 0, Bf, N, 0, P0 == 0 ? 0.0 : 1.0, K, N, 0, 1,
                        0, 0, st));
    }
    symmetrize_kernel<<<(unsigned)((n2 + 255) / 256), 256, 0, st>>>(K, N);
    return hipGetLastError();
}

}  // namespace ri
