// SCF helpers on the GPU: Fock assembly, the DIIS error F D S - S D F and
// extrapolation (Pulay), spectral bounds and trace-correcting purification
// (Niklasson's TC2) giving the projector onto the n_occ lowest orbitals of an
// orthogonalised Fock matrix, and the energy terms.
#include "kernels.h"

#include <algorithm>

namespace {

inline unsigned nb(int64_t n) { int64_t g = (n + 255) / 256; return (unsigned)(g > 1048576 ? 1048576 : g); }

__global__ void fock_kernel(const double* h, const double* J, const double* K, double* F, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        F[i] = h[i] + J[i] - K[i];
}

__global__ void comm_kernel(const double* M, double* e, int N) {
    int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (c >= N) return;
    e[(int64_t)r * N + c] = M[(int64_t)r * N + c] - M[(int64_t)c * N + r];
}

struct Ptrs { const double* p[8]; };

// Two-stage, deterministic reductions over N^2-element matrices: RED_BLOCKS
// workgroups each reduce a fixed grid-stride share into a partial row of
// `red`, then one workgroup combines the partials in order.
constexpr int RED_BLOCKS = 256;

// sum of v over the 256 threads of a workgroup (fixed order)
__device__ __forceinline__ double wg_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

// partial[b][k] = sum over block b's share of x_k * enew (k < m)
__global__ __launch_bounds__(256) void multi_dot_part_kernel(Ptrs es, const double* enew, int m, int64_t n,
                                                             double* red) {
    __shared__ double sh[4];
    double s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) s[k] = 0.0;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double e = enew[i];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < m) s[k] += es.p[k][i] * e;
    }
    for (int k = 0; k < m; ++k) {
        const double t = wg_sum(s[k], sh);
        if (threadIdx.x == 0) red[blockIdx.x * 8 + k] = t;
    }
}

__global__ __launch_bounds__(256) void multi_dot_final_kernel(const double* red, int m, double* row) {
    __shared__ double sh[4];
    for (int k = 0; k < m; ++k) {
        const double t = wg_sum(threadIdx.x < RED_BLOCKS ? red[threadIdx.x * 8 + k] : 0.0, sh);
        if (threadIdx.x == 0) row[k] = t;
    }
}

// Solve [B -1; -1 0] [c; l] = [0; -1] by Gaussian elimination with partial
// pivoting (one thread; m <= 8).
__global__ void diis_solve_kernel(const double* Bm, int m, int ld, double* coef) {
    if (threadIdx.x != 0) return;
    double a[9][10];
    const int n = m + 1;
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < m; ++j) a[i][j] = Bm[i * ld + j];
        a[i][m] = -1.0;
        a[i][n] = 0.0;
    }
    for (int j = 0; j < m; ++j) a[m][j] = -1.0;
    a[m][m] = 0.0;
    a[m][n] = -1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (piv != c)
            for (int k = 0; k <= n; ++k) { double t = a[c][k]; a[c][k] = a[piv][k]; a[piv][k] = t; }
        double d = a[c][c];
        if (d == 0.0) d = 1e-300;
        for (int r = c + 1; r < n; ++r) {
            double f = a[r][c] / d;
            for (int k = c; k <= n; ++k) a[r][k] -= f * a[c][k];
        }
    }
    double x[9];
    for (int r = n - 1; r >= 0; --r) {
        double s = a[r][n];
        for (int k = r + 1; k < n; ++k) s -= a[r][k] * x[k];
        x[r] = s / (a[r][r] == 0.0 ? 1e-300 : a[r][r]);
    }
    for (int i = 0; i < m; ++i) coef[i] = x[i];
}

// DIIS matrix on the device.  row[k] = <e_{slot k}, e_new> for the slots in
// order (the new one last) goes into row and column `snew` of the
// slot-indexed 8 x 8 matrix Bfull; then the m x m matrix of the slots in order
// is gathered into Bm (ld 8) for the solve.  The slot order is host
// bookkeeping that depends on the iteration count only.
struct Slots { int s[8]; };
__global__ void diis_prep_kernel(double* Bfull, const double* row, Slots sl, int m, int snew, double* Bm) {
    if (threadIdx.x == 0)
        for (int k = 0; k < m; ++k) {
            Bfull[snew * 8 + sl.s[k]] = row[k];
            Bfull[sl.s[k] * 8 + snew] = row[k];
        }
    __syncthreads();
    const int i = threadIdx.x >> 3, j = threadIdx.x & 7;
    if (threadIdx.x < 64 && i < m && j < m) Bm[i * 8 + j] = Bfull[sl.s[i] * 8 + sl.s[j]];
}

__global__ void combine_kernel(Ptrs Fs, const double* coef, int m, double* out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += coef[k] * Fs.p[k][i];
        out[i] = s;
    }
}

// Gershgorin interval of each row r (one wave per row): red[2r] = F_rr - sum
// |F_rc|, red[2r + 1] = F_rr + sum |F_rc| over c != r.
__global__ __launch_bounds__(256) void gersh_rows_kernel(const double* F, int N, double* red) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (r >= N) return;
    const double* row = F + (int64_t)r * N;
    double off = 0.0;
    for (int c = lane; c < N; c += 64)
        if (c != r) off += fabs(row[c]);
    for (int o = 32; o > 0; o >>= 1) off += __shfl_down(off, o);
    if (lane == 0) {
        red[2 * r] = row[r] - off;
        red[2 * r + 1] = row[r] + off;
    }
}

__global__ __launch_bounds__(256) void gersh_final_kernel(const double* red, int N, double* bounds) {
    double lo = 1e300, hi = -1e300;
    for (int r = threadIdx.x; r < N; r += 256) {
        lo = fmin(lo, red[2 * r]);
        hi = fmax(hi, red[2 * r + 1]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_down(lo, o));
        hi = fmax(hi, __shfl_down(hi, o));
    }
    __shared__ double sl[4], sh[4];
    if ((threadIdx.x & 63) == 0) { sl[threadIdx.x >> 6] = lo; sh[threadIdx.x >> 6] = hi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        bounds[0] = fmin(fmin(sl[0], sl[1]), fmin(sl[2], sl[3]));
        bounds[1] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    }
}

// Counter-based pseudo-random values in [-1, 1) (a 32-bit integer hash of
// the element index); any full-rank block serves as a subspace start.
__global__ void hash_kernel(double* R, int64_t n, uint32_t seed) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t x = (uint32_t)i * 2654435761u ^ seed;
        x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
        R[i] = (double)x * (2.0 / 4294967296.0) - 1.0;
    }
}

// partial[b] = (D.h, D.J, D.K) over block b's share
__global__ __launch_bounds__(256) void energy_part_kernel(const double* D, const double* h, const double* J,
                                                          const double* K, int64_t n, double* red) {
    __shared__ double sh[4];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double d = D[i];
        a += d * h[i];
        b += d * J[i];
        c += d * K[i];
    }
    a = wg_sum(a, sh);
    b = wg_sum(b, sh);
    c = wg_sum(c, sh);
    if (threadIdx.x == 0) {
        red[blockIdx.x * 3 + 0] = a;
        red[blockIdx.x * 3 + 1] = b;
        red[blockIdx.x * 3 + 2] = c;
    }
}

__global__ __launch_bounds__(256) void energy_final_kernel(const double* red, const double* enuc, double* out) {
    __shared__ double sh[4];
    const bool in = threadIdx.x < RED_BLOCKS;
    const double a = wg_sum(in ? red[threadIdx.x * 3 + 0] : 0.0, sh);
    const double b = wg_sum(in ? red[threadIdx.x * 3 + 1] : 0.0, sh);
    const double c = wg_sum(in ? red[threadIdx.x * 3 + 2] : 0.0, sh);
    if (threadIdx.x == 0) {
        const double en = *enuc;
        out[0] = a + 0.5 * b - 0.5 * c + en;   // E_total
        out[1] = en;
        out[2] = a;                            // E_1e
        out[3] = 0.5 * b;                      // E_J
        out[4] = -0.5 * c;                     // E_K
    }
}

}  // namespace

namespace ri {

hipError_t fock_assemble(const double* h, const double* J, const double* K, double* F, int64_t n, hipStream_t st) {
    fock_kernel<<<nb(n), 256, 0, st>>>(h, J, K, F, n);
    return hipGetLastError();
}
hipError_t commutator(const double* M, double* e, int N, hipStream_t st) {
    comm_kernel<<<dim3((N + 255) / 256, N), 256, 0, st>>>(M, e, N);
    return hipGetLastError();
}
hipError_t diis_dots(const double* const* es, int m, const double* enew, double* row, int64_t n, double* red,
                     hipStream_t st) {
    if (m < 1 || m > 8) return hipErrorInvalidValue;
    Ptrs p{};
    for (int i = 0; i < m; ++i) p.p[i] = es[i];
    multi_dot_part_kernel<<<RED_BLOCKS, 256, 0, st>>>(p, enew, m, n, red);
    RI_TRY(hipGetLastError());
    multi_dot_final_kernel<<<1, 256, 0, st>>>(red, m, row);
    return hipGetLastError();
}
hipError_t diis_prep(double* Bfull, const double* row, const int* slots, int m, int snew, double* Bm,
                     hipStream_t st) {
    if (m < 1 || m > 8) return hipErrorInvalidValue;
    Slots sl{};
    for (int k = 0; k < m; ++k) sl.s[k] = slots[k];
    diis_prep_kernel<<<1, 64, 0, st>>>(Bfull, row, sl, m, snew, Bm);
    return hipGetLastError();
}
hipError_t diis_solve(const double* Bmat, int m, int ld, double* coef, hipStream_t st) {
    diis_solve_kernel<<<1, 64, 0, st>>>(Bmat, m, ld, coef);
    return hipGetLastError();
}
hipError_t diis_combine(const double* const* Fs, const double* coef, int m, double* out, int64_t n, hipStream_t st) {
    Ptrs p{};
    for (int i = 0; i < m; ++i) p.p[i] = Fs[i];
    combine_kernel<<<nb(n), 256, 0, st>>>(p, coef, m, out, n);
    return hipGetLastError();
}
hipError_t gershgorin(const double* F, int N, double* bounds, double* red, hipStream_t st) {
    gersh_rows_kernel<<<(N + 3) / 4, 256, 0, st>>>(F, N, red);
    RI_TRY(hipGetLastError());
    gersh_final_kernel<<<1, 256, 0, st>>>(red, N, bounds);
    return hipGetLastError();
}
hipError_t hash_matrix(double* R, int64_t n, uint32_t seed, hipStream_t st) {
    hash_kernel<<<nb(n), 256, 0, st>>>(R, n, seed);
    return hipGetLastError();
}
hipError_t energy_terms(const double* D, const double* h, const double* J, const double* K, int64_t n,
                        const double* enuc, double* out, double* red, hipStream_t st) {
    energy_part_kernel<<<RED_BLOCKS, 256, 0, st>>>(D, h, J, K, n, red);
    RI_TRY(hipGetLastError());
    energy_final_kernel<<<1, 256, 0, st>>>(red, enuc, out);
    return hipGetLastError();
}

int red_elems(int N) { return std::max(RED_BLOCKS * 8, 2 * N); }

}  // namespace ri
