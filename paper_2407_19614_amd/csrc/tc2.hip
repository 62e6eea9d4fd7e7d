// Trace-correcting purification (Niklasson's TC2) of an orthogonalised Fock
// matrix, one launch per step, for the single-molecule SCF.
//
// A step maps X to X^2 or 2X - X^2, whichever brings the trace closer to
// n_occ, and both need tr X and tr X^2 of the step's input.  X stays exactly
// symmetric (the start is symmetrised and every step forms X X^T, whose
// (i, j) and (j, i) entries are the same products summed in the same order),
// so tr X^2 = sum_ij X_ij^2 is known before the product is formed: each step
// writes, per output tile, the partial sums of tr Y and sum Y_ij^2 of its
// output Y, and every workgroup of the next step sums those partials in one
// fixed order, so all of them take the same branch and the same stopping
// decision.  The stopping rule is the one the batched SCF uses: once
// |tr X - tr X^2| < 1e-11 n_occ, this step and one more run, and later steps
// exit at once, so the host can launch steps in chunks and read the state
// once per chunk instead of once every few steps.  (Near convergence a step
// squares the eigenvalues' distance to 0 or 1 on one side and at most
// doubles it on the other, so the two steps take a summed distance of
// 1e-11 n_occ down to rounding.)
//
// Layout of a step: X^2 is symmetric, so only the upper 48 x 48 output tiles
// are formed (for N = 1000, 231 of them: one workgroup per CU) and each is
// written with its mirror, which keeps X exactly symmetric by construction.
// The eight waves of a workgroup (two per SIMD) take the eighths of the
// reduction index; each wave owns the whole tile as 3 x 3 FP64 MFMA tiles
// and reads its operands straight from X: the A operand of row tile i is
// X[k][m0 + 16 i + ..] (a row of X, by symmetry) and the B operand of
// column tile j is X[k][n0 + 16 j + ..], so the 16 lanes of each group read
// 16 consecutive doubles.  Buffer loads return zero past the end of X (rows
// k >= N), and the operands of the k-step four ahead are in flight while a
// step's 9 MFMAs run.  The eight partial tiles are summed through LDS in one
// fixed order, then the update, the tile and mirror writes and the partial
// sums run in the epilogue.
#include "kernels.h"

#include <algorithm>
#include <climits>

namespace {

constexpr int TT = 48;        // output tile edge (3 MFMA tiles)
constexpr int LDT = TT + 1;   // padded LDS row
constexpr int PD = 4;         // k-steps of operands in flight

__host__ __device__ inline int n_tiles_edge(int N) { return (N + TT - 1) / TT; }

// upper tile t (row-major over I <= J) of an nt x nt tiling
__device__ inline void upper_tile48(int t, int nt, int& I, int& J) {
    int i = 0, rem = t;
    while (rem >= nt - i) {
        rem -= nt - i;
        ++i;
    }
    I = i;
    J = i + rem;
}

// state fields (int[8] per parity buffer)
constexpr int S_CD = 0, S_DONE = 1, S_STEPS = 2, S_LAST = 3;

// sum of v over the NT threads of the workgroup, in a fixed order
template <int NT>
__device__ __forceinline__ double wg_sum_fixed(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += sh[i];
    return r;
}

// X0 = (hi I - (F + F^T)/2) / (hi - lo) on the upper 48 x 48 tiles (each
// written with its mirror), with each tile's partial sums of tr X0 and
// sum X0_ij^2 over the entries it stands for, and the purification state
// reset.
__global__ __launch_bounds__(256) void tc2f_init_kernel(const double* __restrict__ F,
                                                        const double* __restrict__ bounds, int N,
                                                        double* __restrict__ X, double* __restrict__ part,
                                                        int* __restrict__ st) {
    __shared__ double sh[4];
    const int nt = n_tiles_edge(N);
    int I, J;
    upper_tile48(blockIdx.x, nt, I, J);
    const double lo = bounds[0], hi = bounds[1], s = 1.0 / (hi - lo);
    double f2 = 0.0, tr = 0.0;
    for (int e = threadIdx.x; e < TT * TT; e += 256) {
        const int r = TT * I + e / TT, c = TT * J + e % TT;
        if (r < N && c < N) {
            const double fs = 0.5 * (F[(int64_t)r * N + c] + F[(int64_t)c * N + r]);
            const double x = ((r == c ? hi : 0.0) - fs) * s;
            X[(int64_t)r * N + c] = x;
            if (I != J) X[(int64_t)c * N + r] = x;
            f2 += (I == J ? 1.0 : 2.0) * x * x;
            if (r == c) tr += x;
        }
    }
    tr = wg_sum_fixed<256>(tr, sh);
    f2 = wg_sum_fixed<256>(f2, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = tr;
        part[2 * blockIdx.x + 1] = f2;
    }
    if (blockIdx.x == 0 && threadIdx.x < 8) st[threadIdx.x] = threadIdx.x == S_CD ? -1 : 0;
}

// One wave's share of a 48 x 48 tile of X^2: k-steps kbeg + 4 s, s < nks,
// as 3 x 3 MFMA tiles (DIAG: the row and column panels coincide).  Buffer
// loads over X with the whole offset in the lane's offset, so that rows
// k >= N read as zero (range check) and the prefetch past the last k-step
// stays inside the check.
template <bool DIAG>
__device__ __forceinline__ void tc2_accumulate(const double* X, int N, int kbeg, int nks, int m0, int n0, int r,
                                               int g, d4_t (&acc)[3][3]) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X), (short)0, N * N * 8, 0x00020000);
    int vA[3], vB[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        vA[i] = ((kbeg + g) * N + m0 + 16 * i + r) * 8;
        vB[i] = ((kbeg + g) * N + n0 + 16 * i + r) * 8;
    }
    const int step = 4 * N * 8;
    auto ld = [&](int s, double (&pa)[3], double (&pb)[3]) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
            pa[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, vA[i] + s * step, 0, 0));
        if (!DIAG) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
                pb[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, vB[i] + s * step, 0, 0));
        }
    };
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
    double pa[PD][3], pb[PD][3];
#pragma unroll
    for (int p = 0; p < PD; ++p) ld(p, pa[p], pb[p]);
    for (int s0 = 0; s0 < nks; s0 += PD) {
#pragma unroll
        for (int p = 0; p < PD; ++p) {
            if (s0 + p < nks) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) acc[i][j] = mfma_f64(pa[p][i], DIAG ? pa[p][j] : pb[p][j], acc[i][j]);
                ld(s0 + p + PD, pa[p], pb[p]);
            }
        }
    }
}

__global__ __launch_bounds__(512) void tc2f_step_kernel(const double* __restrict__ X, double* __restrict__ Y, int N,
                                                        int n_occ, const double* __restrict__ part_in,
                                                        double* __restrict__ part_out, const int* __restrict__ st_in,
                                                        int* __restrict__ st_out, int out_id) {
    __shared__ double sh[8];
    __shared__ double red[4][TT][LDT];   // partial tiles: waves w and w + 4 in slot w
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nt = n_tiles_edge(N), tiles = nt * (nt + 1) / 2;
    if (st_in[S_DONE]) {
        if (blockIdx.x == 0 && tid < 8) st_out[tid] = st_in[tid];
        return;
    }
    // tr X and tr X^2 from the previous step's partial sums (same order everywhere)
    double a = 0.0, b = 0.0;
    for (int i = tid; i < tiles; i += 512) {
        a += part_in[2 * i];
        b += part_in[2 * i + 1];
    }
    const double t1 = wg_sum_fixed<512>(a, sh);
    const double t2 = wg_sum_fixed<512>(b, sh);
    int cd = st_in[S_CD];
    if (cd < 0) {
        if (fabs(t1 - t2) < 1e-11 * (double)max(1, n_occ)) cd = 1;
    } else if (cd > 0) {
        --cd;
    }
    const bool sq = fabs(t2 - n_occ) < fabs(2.0 * t1 - t2 - n_occ);
    if (blockIdx.x == 0 && tid == 0) {
        st_out[S_CD] = cd;
        st_out[S_DONE] = cd == 0;                 // this step's update is the last
        st_out[S_STEPS] = st_in[S_STEPS] + 1;
        st_out[S_LAST] = out_id;
        for (int k = 4; k < 8; ++k) st_out[k] = st_in[k];
    }
    const int L = xcd_remap(blockIdx.x, tiles);
    int I, J;
    upper_tile48(L, nt, I, J);
    const int m0 = TT * I, n0 = TT * J;
    const bool diag = I == J;
    // this wave's eighth of the reduction index, in whole 4-deep k-steps
    const int Kq = ((N + 7) / 8 + 3) / 4 * 4;
    const int kbeg = wave * Kq, kend = min(N, kbeg + Kq), nks = max(0, (kend - kbeg + 3) / 4);
    const int r = lane & 15, g = lane >> 4;
    d4_t acc[3][3];
    if (diag) tc2_accumulate<true>(X, N, kbeg, nks, m0, n0, r, g, acc);
    else tc2_accumulate<false>(X, N, kbeg, nks, m0, n0, r, g, acc);
    // partial tiles to LDS: element q of lane (c, g) in MFMA tile (i, j) is
    // row 16 i + 4 q + g, column 16 j + c.  Waves 4-7 write slot w - 4, then
    // waves 0-3 add theirs to slot w (each lane to the entries it wrote).
    if (wave >= 4) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) red[wave - 4][16 * i + 4 * q + g][16 * j + r] = acc[i][j][q];
    }
    __syncthreads();
    if (wave < 4) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) red[wave][16 * i + 4 * q + g][16 * j + r] += acc[i][j][q];
    }
    __syncthreads();
    // sum of the slots in one fixed order, the update, the tile's write
    // (diagonal tiles: the upper triangle) and the partial sums; for 2X - X^2
    // the entries of X are loaded, from clamped addresses, before the first
    // store
    constexpr int EP = (TT * TT + 511) / 512;
    double xo[EP];
    if (!sq) {
#pragma unroll
        for (int t = 0; t < EP; ++t) {
            const int e = min(tid + 512 * t, TT * TT - 1), gm = min(m0 + e / TT, N - 1), gn = min(n0 + e % TT, N - 1);
            xo[t] = X[(int64_t)gm * N + gn];
        }
    }
    double f2 = 0.0, tr = 0.0;
#pragma unroll
    for (int t = 0; t < EP; ++t) {
        const int e = tid + 512 * t;
        if (e < TT * TT) {
            const int rr = e / TT, cc = e % TT, gm = m0 + rr, gn = n0 + cc;
            double v = 0.0;
            if (gm < N && gn < N && (!diag || rr <= cc)) {
                const double x2 = ((red[0][rr][cc] + red[1][rr][cc]) + red[2][rr][cc]) + red[3][rr][cc];
                v = sq ? x2 : 2.0 * xo[t] - x2;
                Y[(int64_t)gm * N + gn] = v;
                f2 += (gm == gn ? 1.0 : 2.0) * v * v;
                if (gm == gn) tr += v;
            }
            red[0][rr][cc] = v;   // each element is read and rewritten by one thread
        }
    }
    __syncthreads();
    // mirror: Y[n][m] = Y[m][n], read transposed from LDS so that the writes
    // run along rows of Y
#pragma unroll
    for (int t = 0; t < EP; ++t) {
        const int e = tid + 512 * t;
        if (e < TT * TT) {
            const int cc = e / TT, rr = e % TT, gm = m0 + rr, gn = n0 + cc;
            if (gm < N && gn < N && (diag ? rr < cc : true)) Y[(int64_t)gn * N + gm] = red[0][rr][cc];
        }
    }
    tr = wg_sum_fixed<512>(tr, sh);
    f2 = wg_sum_fixed<512>(f2, sh);
    if (tid == 0) {
        part_out[2 * L] = tr;
        part_out[2 * L + 1] = f2;
    }
}

// The latest X is in Y when the last step that ran wrote there: copy it back.
__global__ void tc2f_final_kernel(double* X, const double* Y, int64_t n, const int* st) {
    if (st[S_LAST] != 1) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        X[i] = Y[i];
}

}  // namespace

namespace ri {

int tc2f_tiles(int N) {
    const int nt = n_tiles_edge(N);
    return nt * (nt + 1) / 2;
}

hipError_t tc2f_init(const double* F, const double* bounds, int N, double* X, double* part, int* state,
                     hipStream_t st) {
    tc2f_init_kernel<<<tc2f_tiles(N), 256, 0, st>>>(F, bounds, N, X, part, state);
    return hipGetLastError();
}

hipError_t tc2f_step(const double* X, double* Y, int N, int n_occ, const double* part_in, double* part_out,
                     const int* st_in, int* st_out, int out_id, hipStream_t st) {
    // buffer offsets into X, including the prefetch past the last k-step, are 32-bit
    if ((int64_t)(N + 4 * PD + 8) * N * 8 > INT_MAX) return hipErrorInvalidValue;
    tc2f_step_kernel<<<tc2f_tiles(N), 512, 0, st>>>(X, Y, N, n_occ, part_in, part_out, st_in, st_out, out_id);
    return hipGetLastError();
}

hipError_t tc2f_final(double* X, const double* Y, int N, const int* state, hipStream_t st) {
    const int64_t n = (int64_t)N * N;
    const int64_t g = std::min<int64_t>((n + 255) / 256, 4096);
    tc2f_final_kernel<<<(unsigned)g, 256, 0, st>>>(X, Y, n, state);
    return hipGetLastError();
}

}  // namespace ri
