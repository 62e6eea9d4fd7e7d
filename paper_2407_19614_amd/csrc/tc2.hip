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
// Layout of a step: 64 x 64 output tiles, one workgroup of 8 waves each.
// Waves 0-3 and 4-7 take the two halves of the reduction index (split-K
// inside the workgroup), each half staging 16-deep slices of the tile's
// row panel X[64I .., :] and column panel X[64J .., :] (rows of X, by
// symmetry) through a double-buffered LDS ring with one barrier per slice;
// each wave owns a 32 x 32 quadrant (2 x 2 FP64 MFMA tiles).  The second
// half's accumulators are added through LDS, then the update, the output
// write and the partial sums run in the epilogue.
#include "kernels.h"

#include <algorithm>

namespace {

constexpr int TT = 64;        // output tile edge
constexpr int SK = 16;        // slice depth
constexpr int LDT = TT + 1;   // padded LDS row

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

// X0 = (hi I - (F + F^T)/2) / (hi - lo) on 64 x 64 tiles, with each tile's
// partial sums of tr X0 and sum X0_ij^2, and the purification state reset.
__global__ __launch_bounds__(256) void tc2f_init_kernel(const double* __restrict__ F,
                                                        const double* __restrict__ bounds, int N,
                                                        double* __restrict__ X, double* __restrict__ part,
                                                        int* __restrict__ st) {
    __shared__ double sh[4];
    const int nt = (N + TT - 1) / TT, I = blockIdx.x / nt, J = blockIdx.x % nt;
    const double lo = bounds[0], hi = bounds[1], s = 1.0 / (hi - lo);
    double f2 = 0.0, tr = 0.0;
    for (int e = threadIdx.x; e < TT * TT; e += 256) {
        const int r = TT * I + (e >> 6), c = TT * J + (e & 63);
        if (r < N && c < N) {
            const double fs = 0.5 * (F[(int64_t)r * N + c] + F[(int64_t)c * N + r]);
            const double x = ((r == c ? hi : 0.0) - fs) * s;
            X[(int64_t)r * N + c] = x;
            f2 += x * x;
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

__global__ __launch_bounds__(512) void tc2f_step_kernel(const double* __restrict__ X, double* __restrict__ Y, int N,
                                                        int n_occ, const double* __restrict__ part_in,
                                                        double* __restrict__ part_out, const int* __restrict__ st_in,
                                                        int* __restrict__ st_out, int out_id) {
    __shared__ double sh[8];
    __shared__ double As[2][2][SK][LDT];   // [half][stage][k][row]
    __shared__ double Bs[2][2][SK][LDT];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, half = wave >> 2, w4 = wave & 3;
    const int nt = (N + TT - 1) / TT, tiles = nt * nt;
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
    const int m0 = TT * (L / nt), n0 = TT * (L % nt);
    // reduction halves, rounded to whole slices
    const int Kh = min(N, ((N + 1) / 2 + SK - 1) / SK * SK);
    const int kb = half ? Kh : 0, ke = half ? N : Kh;
    const int nsl = (max(Kh, N - Kh) + SK - 1) / SK;   // the same count in both halves
    // loader lanes: 256 per half; element gt + 256 i of the 64 x SK slice is
    // row (gt + 256 i) / SK, k = gt % SK, so SK consecutive lanes read one
    // row's SK consecutive doubles (whole cache lines per instruction)
    constexpr int KQ = SK / 4, RS = 256 / SK;
    const int gt = tid & 255, lk0 = gt % SK, lr0 = gt / SK;
    double ra[KQ], rb[KQ];
    // unconditional loads from clamped addresses, zeroed by a select only
    // when they are stored (no branch around each load, and no wait for the
    // load before the MFMAs of the current slice)
    bool kin = false;
    auto load = [&](int s) {
        const int k = kb + s * SK + lk0;
        kin = k < ke;
        const int kc = min(k, N - 1);
#pragma unroll
        for (int i = 0; i < KQ; ++i) {
            const int r = lr0 + RS * i;
            ra[i] = X[(int64_t)min(m0 + r, N - 1) * N + kc];
            rb[i] = X[(int64_t)min(n0 + r, N - 1) * N + kc];
        }
    };
    auto store = [&](int stg) {
#pragma unroll
        for (int i = 0; i < KQ; ++i) {
            const int r = lr0 + RS * i;
            As[half][stg][lk0][r] = (kin && m0 + r < N) ? ra[i] : 0.0;
            Bs[half][stg][lk0][r] = (kin && n0 + r < N) ? rb[i] : 0.0;
        }
    };
    d4_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
    const int wm = (w4 >> 1) * 32, wn = (w4 & 1) * 32, li = lane & 15, lk = lane >> 4;
    load(0);
    store(0);
    __syncthreads();
    for (int s = 0; s < nsl; ++s) {
        const int cur = s & 1;
        if (s + 1 < nsl) load(s + 1);
        // operands of the next k-step are read from LDS before this step's
        // MFMAs, so their latency hides under the MFMAs
        double a0 = As[half][cur][lk][wm + li], a1 = As[half][cur][lk][wm + 16 + li];
        double b0 = Bs[half][cur][lk][wn + li], b1 = Bs[half][cur][lk][wn + 16 + li];
#pragma unroll
        for (int kk = 0; kk < SK; kk += 4) {
            double na0 = 0.0, na1 = 0.0, nb0 = 0.0, nb1 = 0.0;
            if (kk + 4 < SK) {
                na0 = As[half][cur][kk + 4 + lk][wm + li];
                na1 = As[half][cur][kk + 4 + lk][wm + 16 + li];
                nb0 = Bs[half][cur][kk + 4 + lk][wn + li];
                nb1 = Bs[half][cur][kk + 4 + lk][wn + 16 + li];
            }
            __builtin_amdgcn_sched_barrier(0);   // keep those reads ahead of the MFMAs
            acc[0][0] = mfma_f64(a0, b0, acc[0][0]);
            acc[0][1] = mfma_f64(a0, b1, acc[0][1]);
            acc[1][0] = mfma_f64(a1, b0, acc[1][0]);
            acc[1][1] = mfma_f64(a1, b1, acc[1][1]);
            a0 = na0; a1 = na1; b0 = nb0; b1 = nb1;
        }
        if (s + 1 < nsl) store(cur ^ 1);
        __syncthreads();
    }
    // second half's sums through LDS (the ring is free now: 4 x 16 rows of 65)
    double (*R)[LDT] = reinterpret_cast<double (*)[LDT]>(&As[0][0][0][0]);
    if (half == 1) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) R[wm + 16 * i + 4 * r + lk][wn + 16 * j + li] = acc[i][j][r];
    }
    __syncthreads();
    double f2 = 0.0, tr = 0.0;
    if (half == 0) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = wm + 16 * i + 4 * r + lk, cc = wn + 16 * j + li;
                    const int gm = m0 + rr, gn = n0 + cc;
                    if (gm < N && gn < N) {
                        const double x2 = acc[i][j][r] + R[rr][cc];
                        const int64_t idx = (int64_t)gm * N + gn;
                        const double v = sq ? x2 : 2.0 * X[idx] - x2;
                        Y[idx] = v;
                        f2 += v * v;
                        if (gm == gn) tr += v;
                    }
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
    const int nt = (N + TT - 1) / TT;
    return nt * nt;
}

hipError_t tc2f_init(const double* F, const double* bounds, int N, double* X, double* part, int* state,
                     hipStream_t st) {
    tc2f_init_kernel<<<tc2f_tiles(N), 256, 0, st>>>(F, bounds, N, X, part, state);
    return hipGetLastError();
}

hipError_t tc2f_step(const double* X, double* Y, int N, int n_occ, const double* part_in, double* part_out,
                     const int* st_in, int* st_out, int out_id, hipStream_t st) {
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
