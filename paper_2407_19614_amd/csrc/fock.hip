// RI Fock build: decompression of the fitted tensor into packed symmetric
// tiles, the exchange half-transform X^P = B^P C_occ on MFMA, the exchange
// SYRK K = sum_P X^P X^P^T over lower tiles with split-K, and the
// bandwidth-bound Coulomb contractions gamma = B:D, J = sum_P gamma_P B^P on
// the compressed (significant-pair) tensor.
#include "kernels.h"

#include <algorithm>

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

// B[P][tile][r*64+c] = Bc[P][pair(64I+r, 64J+c)] or 0, for PB consecutive P
// per workgroup so that each pair-map lookup serves all of them.
constexpr int PACK_PB = 4;
template <typename T>
__global__ __launch_bounds__(256) void pack_kernel(const double* Bc, int64_t n_pairs, const int32_t* map,
                                                   int N, int64_t ntl, int n_aux, T* B) {
    const int t = blockIdx.x, P0 = blockIdx.y * PACK_PB;
    int I, J;
    tile_ij(t, I, J);
    for (int e = threadIdx.x; e < 4096; e += 256) {
        const int mu = 64 * I + (e >> 6), nu = 64 * J + (e & 63);
        int32_t q = -1;
        if (mu < N && nu < N) q = map[(int64_t)max(mu, nu) * N + min(mu, nu)];
#pragma unroll
        for (int p = 0; p < PACK_PB; ++p) {
            const int P = P0 + p;
            if (P < n_aux) B[((int64_t)P * ntl + t) * 4096 + e] = (T)(q >= 0 ? Bc[(int64_t)P * n_pairs + q] : 0.0);
        }
    }
}

// X^T for (row-block I, auxiliary pair P0, P0+1): each wave owns one P and
// 32 columns mu (2 MFMA column tiles) over MF full 16-row occupied tiles and
// TQ trailing 4-row quads, so the staged C_occ slice serves both P.  The
// quads run on the 4-block 4x4x4 FP64 MFMA, whose B operand takes the same
// lane mapping as the 16x16x4 one (block = lane/4 % 4 covers columns
// 4*block .. 4*block+3 of the 16), so a row count that is not a multiple of
// 16 does not pay for a whole padded tile: one quad costs a quarter of a
// 16x16x4 issue.  Next-slice global loads are held in registers while the
// current slice is multiplied, issued between the first two k-steps so the
// MFMA pipe is not left idle while they go out.
//
// CPAD: C is the zero-padded copy [64 * nt rows][cld >= i0 + 16*ceil(W/16)],
// so every load is unconditional, and loads go through buffer resources;
// otherwise C is [N][n_occ] with bounds tests.  With a single auxiliary index left (P0 + 1 == n_aux) the second
// half reads P0's tiles again and its results are not stored.  TB is the
// storage type of B: double, or float widened exactly to FP64 on load (the
// products and sums stay FP64).
template <int MF, int TQ, bool CPAD, typename TB = double>
__device__ __forceinline__ void x2_body_f64(int I, int P0, int i0, const TB* __restrict__ B, int nt, int64_t ntl,
                                            const double* __restrict__ C, int cld, int N, int n_occ, int n_aux,
                                            double* __restrict__ Xt, int Npad) {
    constexpr int W = MF * 16 + TQ * 4;            // occupied columns used per slice
    constexpr int WS = CPAD ? (W + 15) / 16 * 16 : W;   // columns staged per slice
    constexpr int NCR = (16 * WS + 255) / 256;     // C elements per thread per slice
    __shared__ double Bs[2][16][65];
    __shared__ double Cs[16][WS + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int ps = wave >> 1, h = wave & 1;
    const TB* Bp0 = B + (int64_t)P0 * ntl * 4096;
    const TB* Bp1 = B + (int64_t)(P0 + 1 < n_aux ? P0 + 1 : P0) * ntl * 4096;
    constexpr int EB = sizeof(TB);                 // bytes per stored B element
    double rb[8], rc[NCR];
#if defined(__HIP_DEVICE_COMPILE__)
    // CPAD form: buffer loads whose lane offsets are fixed per orientation
    // and whose slice offset is a scalar, so a slice's loads need no vector
    // address arithmetic.  One auxiliary index's tiles span ntl * 32 KiB.
    __amdgpu_buffer_rsrc_t rs0, rs1, rsc;
    int boffL[4], boffU[4], coff[NCR];
    if constexpr (CPAD) {
        const int tb = (int)(ntl * 4096 * EB);
        rs0 = __builtin_amdgcn_make_buffer_rsrc(const_cast<TB*>(Bp0), (short)0, tb, 0x00020000);
        rs1 = __builtin_amdgcn_make_buffer_rsrc(const_cast<TB*>(Bp1), (short)0, tb, 0x00020000);
        rsc = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(C), (short)0, nt * 64 * cld * 8, 0x00020000);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            boffL[r] = (((tid >> 4) + 16 * r) * 64 + (tid & 15)) * EB;    // tile row m, column k
            boffU[r] = (((tid >> 6) + 4 * r) * 64 + (tid & 63)) * EB;     // tile row k, column m
        }
#pragma unroll
        for (int r = 0; r < NCR; ++r) {
            const int e = tid + 256 * r;
            coff[r] = ((e / WS) * cld + e % WS) * 8;
        }
    }
    auto ldb = [](__amdgpu_buffer_rsrc_t rs, int vo, int so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, 0));
    };
    // a B element in FP64 (FP32 storage is widened exactly)
    auto ldbt = [](__amdgpu_buffer_rsrc_t rs, int vo, int so) -> double {
        if constexpr (EB == 8)
            return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, 0));
        else
            return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0));
    };
#endif
    auto load_b = [&](int J, int k0) {
        const bool lower = J <= I;
        const int tile = lower ? (I * (I + 1) / 2 + J) : (J * (J + 1) / 2 + I);
        if constexpr (CPAD) {
#if defined(__HIP_DEVICE_COMPILE__)
            if (lower) {
                const int so = (tile * 4096 + k0) * EB;
#pragma unroll
                for (int r = 0; r < 4; ++r) { rb[r] = ldbt(rs0, boffL[r], so); rb[4 + r] = ldbt(rs1, boffL[r], so); }
            } else {
                const int so = (tile * 4096 + k0 * 64) * EB;
#pragma unroll
                for (int r = 0; r < 4; ++r) { rb[r] = ldbt(rs0, boffU[r], so); rb[4 + r] = ldbt(rs1, boffU[r], so); }
            }
#endif
        } else {
            const int64_t toff = (int64_t)tile * 4096;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int off;
                if (lower) { int k = tid & 15, m = (tid >> 4) + 16 * r; off = m * 64 + k0 + k; }
                else       { int m = tid & 63, k = (tid >> 6) + 4 * r; off = (k0 + k) * 64 + m; }
                rb[r] = Bp0[toff + off];
                rb[4 + r] = Bp1[toff + off];
            }
        }
    };
    auto load_c = [&](int J, int k0) {
        if constexpr (CPAD) {
#if defined(__HIP_DEVICE_COMPILE__)
            const int so = ((64 * J + k0) * cld + i0) * 8;
#pragma unroll
            for (int r = 0; r < NCR; ++r)
                if (16 * WS % 256 == 0 || tid + 256 * r < 16 * WS) rc[r] = ldb(rsc, coff[r], so);
#endif
        } else {
#pragma unroll
            for (int r = 0; r < NCR; ++r) {
                int e = tid + 256 * r, k = e / WS, i = e % WS;
                int nu = 64 * J + k0 + k, gi = i0 + i;
                rc[r] = (e < 16 * WS && nu < N && gi < n_occ) ? C[(int64_t)nu * n_occ + gi] : 0.0;
            }
        }
    };
    auto store = [&](int J) {
        const bool lower = J <= I;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int k, m;
            if (lower) { k = tid & 15; m = (tid >> 4) + 16 * r; }
            else       { m = tid & 63; k = (tid >> 6) + 4 * r; }
            Bs[0][k][m] = rb[r];
            Bs[1][k][m] = rb[4 + r];
        }
#pragma unroll
        for (int r = 0; r < NCR; ++r) {
            int e = tid + 256 * r;
            if (16 * WS % 256 == 0 || e < 16 * WS) Cs[e / WS][e % WS] = rc[r];
        }
    };
    d4_t acc[MF > 0 ? MF : 1][2];
    double accq[TQ > 0 ? TQ : 1][2];
#pragma unroll
    for (int m = 0; m < MF; ++m) { acc[m][0] = d4_t{0, 0, 0, 0}; acc[m][1] = d4_t{0, 0, 0, 0}; }
#pragma unroll
    for (int q = 0; q < TQ; ++q) { accq[q][0] = 0.0; accq[q][1] = 0.0; }
    const int nsl = (N + 15) / 16;                 // 16-deep k-slices that hold a basis function
    load_b(0, 0);
    load_c(0, 0);
    for (int sl = 0; sl < nsl; ++sl) {
        const int J = sl >> 2;
        __syncthreads();
        store(J);
        __syncthreads();
        const bool more = sl + 1 < nsl;
        const int Jn = (sl + 1) >> 2, kn = ((sl + 1) & 3) * 16;
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            double b0 = Bs[ps][kk + lk][h * 32 + li], b1 = Bs[ps][kk + lk][h * 32 + 16 + li];
#pragma unroll
            for (int m = 0; m < MF; ++m) {
                double a = Cs[kk + lk][m * 16 + li];
                acc[m][0] = mfma_f64(a, b0, acc[m][0]);
                acc[m][1] = mfma_f64(a, b1, acc[m][1]);
            }
            // 4x4x4 block operands: A row = lane % 4, k = lane / 16
#pragma unroll
            for (int q = 0; q < TQ; ++q) {
                double a = Cs[kk + lk][MF * 16 + 4 * q + (lane & 3)];
                accq[q][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b0, accq[q][0], 0, 0, 0);
                accq[q][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b1, accq[q][1], 0, 0, 0);
            }
            if (kk == 0 && more) load_b(Jn, kn);
            if (kk == 4 && more) load_c(Jn, kn);
        }
    }
    const int P = P0 + ps;
    if (P >= n_aux) return;
#pragma unroll
    for (int m = 0; m < MF; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int i = i0 + m * 16 + 4 * r + lk;
                if (i < n_occ) Xt[((int64_t)P * n_occ + i) * Npad + 64 * I + h * 32 + n * 16 + li] = acc[m][n][r];
            }
    // 4x4x4 result: row = lane / 16, column = lane % 16 (block-major)
#pragma unroll
    for (int q = 0; q < TQ; ++q)
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            int i = i0 + MF * 16 + 4 * q + lk;
            if (i < n_occ) Xt[((int64_t)P * n_occ + i) * Npad + 64 * I + h * 32 + n * 16 + li] = accq[q][n];
        }
}

template <int MF, int TQ, typename TB = double>
__global__ __launch_bounds__(256, 2) void x2_kernel_f64(const TB* __restrict__ B, int nt, int64_t ntl,
                                                     const double* __restrict__ Cp, int cld, int N, int n_occ,
                                                     int n_aux, double* __restrict__ Xt, int Npad) {
    const int L = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    x2_body_f64<MF, TQ, true, TB>(L % gridDim.x, 2 * (L / gridDim.x), blockIdx.z * 128, B, nt, ntl, Cp, cld, N,
                                  n_occ, n_aux, Xt, Npad);
}


__global__ void cpad_kernel(const double* C, int N, int n_occ, int rows, int cld, double* Cp) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cld) return;
    int r = e / cld, c = e % cld;
    Cp[e] = (r < N && c < n_occ) ? C[(int64_t)r * n_occ + c] : 0.0;
}

// FP32 forms of the exchange contractions (precision extension): B in FP32,
// v_mfma_f32_16x16x4f32 (lane l holds D[4*(l/16) + r][l%16]), X in FP32.
__device__ __forceinline__ f4_t mfma_f32(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int MT, bool CPAD>
__device__ __forceinline__ void x2_body_f32(int I, int P0, int i0, const float* __restrict__ B, int nt, int64_t ntl,
                                            const double* __restrict__ C, const float* __restrict__ Cf, int cld,
                                            int N, int n_occ, int n_aux, float* __restrict__ Xt, int Npad) {
    // CPAD: C_occ arrives as the FP32 zero-padded copy Cf [64 * nt][cld] and
    // every load goes through a buffer resource (as in the FP64 form);
    // otherwise C is FP64 [N][n_occ] with bounds tests.
    constexpr int W = MT * 16;
    __shared__ float Bs[2][16][65];
    __shared__ float Cs[16][W + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int ps = wave >> 1, h = wave & 1;
    const float* Bp0 = B + (int64_t)P0 * ntl * 4096;
    const float* Bp1 = B + (int64_t)(P0 + 1 < n_aux ? P0 + 1 : P0) * ntl * 4096;
    float rb[8], rc[MT];
#if defined(__HIP_DEVICE_COMPILE__)
    __amdgpu_buffer_rsrc_t rs0, rs1, rsc;
    int boffL[4], boffU[4], coff[MT];
    if constexpr (CPAD) {
        const int tb = (int)(ntl * 4096 * 4);
        rs0 = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(Bp0), (short)0, tb, 0x00020000);
        rs1 = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(Bp1), (short)0, tb, 0x00020000);
        rsc = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(Cf), (short)0, nt * 64 * cld * 4, 0x00020000);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            boffL[r] = (((tid >> 4) + 16 * r) * 64 + (tid & 15)) * 4;
            boffU[r] = (((tid >> 6) + 4 * r) * 64 + (tid & 63)) * 4;
        }
#pragma unroll
        for (int r = 0; r < MT; ++r) {
            const int e = tid + 256 * r;
            coff[r] = ((e / W) * cld + e % W) * 4;
        }
    }
    auto ldf = [](__amdgpu_buffer_rsrc_t rs, int vo, int so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0));
    };
#endif
    auto load_b = [&](int J, int k0) {
        const bool lower = J <= I;
        const int tile = lower ? (I * (I + 1) / 2 + J) : (J * (J + 1) / 2 + I);
        if constexpr (CPAD) {
#if defined(__HIP_DEVICE_COMPILE__)
            if (lower) {
                const int so = (tile * 4096 + k0) * 4;
#pragma unroll
                for (int r = 0; r < 4; ++r) { rb[r] = ldf(rs0, boffL[r], so); rb[4 + r] = ldf(rs1, boffL[r], so); }
            } else {
                const int so = (tile * 4096 + k0 * 64) * 4;
#pragma unroll
                for (int r = 0; r < 4; ++r) { rb[r] = ldf(rs0, boffU[r], so); rb[4 + r] = ldf(rs1, boffU[r], so); }
            }
#endif
        } else {
            const int64_t toff = (int64_t)tile * 4096;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int off;
                if (lower) { int k = tid & 15, m = (tid >> 4) + 16 * r; off = m * 64 + k0 + k; }
                else       { int m = tid & 63, k = (tid >> 6) + 4 * r; off = (k0 + k) * 64 + m; }
                rb[r] = Bp0[toff + off];
                rb[4 + r] = Bp1[toff + off];
            }
        }
    };
    auto load_c = [&](int J, int k0) {
        if constexpr (CPAD) {
#if defined(__HIP_DEVICE_COMPILE__)
            const int so = ((64 * J + k0) * cld + i0) * 4;
#pragma unroll
            for (int r = 0; r < MT; ++r) rc[r] = ldf(rsc, coff[r], so);
#endif
        } else {
#pragma unroll
            for (int r = 0; r < MT; ++r) {
                int e = tid + 256 * r, k = e / W, i = e % W;
                int nu = 64 * J + k0 + k, gi = i0 + i;
                rc[r] = (nu < N && gi < n_occ) ? (float)C[(int64_t)nu * n_occ + gi] : 0.0f;
            }
        }
    };
    auto store = [&](int J) {
        const bool lower = J <= I;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int k, m;
            if (lower) { k = tid & 15; m = (tid >> 4) + 16 * r; }
            else       { m = tid & 63; k = (tid >> 6) + 4 * r; }
            Bs[0][k][m] = rb[r];
            Bs[1][k][m] = rb[4 + r];
        }
#pragma unroll
        for (int r = 0; r < MT; ++r) {
            int e = tid + 256 * r;
            Cs[e / W][e % W] = rc[r];
        }
    };
    f4_t acc[MT][2];
    d4_t acc64[MT][2];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        acc[m][0] = acc[m][1] = f4_t{0, 0, 0, 0};
        acc64[m][0] = acc64[m][1] = d4_t{0, 0, 0, 0};
    }
    const int nsl = (N + 15) / 16;                 // 16-deep k-slices that hold a basis function
    load_b(0, 0);
    load_c(0, 0);
    for (int sl = 0; sl < nsl; ++sl) {
        const int J = sl >> 2;
        __syncthreads();
        store(J);
        __syncthreads();
        const bool more = sl + 1 < nsl;
        const int Jn = (sl + 1) >> 2, kn = ((sl + 1) & 3) * 16;
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            float b0 = Bs[ps][kk + lk][h * 32 + li], b1 = Bs[ps][kk + lk][h * 32 + 16 + li];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                float a = Cs[kk + lk][m * 16 + li];
                acc[m][0] = mfma_f32(a, b0, acc[m][0]);
                acc[m][1] = mfma_f32(a, b1, acc[m][1]);
            }
            if (kk == 0 && more) load_b(Jn, kn);
            if (kk == 4 && more) load_c(Jn, kn);
        }
        if ((sl & 3) == 3 || !more) {   // FP32 over one 64-wide nu tile, FP64 across tiles
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int n = 0; n < 2; ++n)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        acc64[m][n][r] += (double)acc[m][n][r];
                        acc[m][n][r] = 0.0f;
                    }
        }
    }
    const int P = P0 + ps;
    if (P >= n_aux) return;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int i = i0 + m * 16 + 4 * lk + r;
                if (i < n_occ) Xt[((int64_t)P * n_occ + i) * Npad + 64 * I + h * 32 + n * 16 + li] = (float)acc64[m][n][r];
            }
}

template <int MT>
__global__ __launch_bounds__(256, 2) void x2_kernel_f32(const float* __restrict__ B, int nt, int64_t ntl,
                                                        const float* __restrict__ Cf, int cld, int N, int n_occ,
                                                        int n_aux, float* __restrict__ Xt, int Npad) {
    const int L = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    x2_body_f32<MT, true>(L % gridDim.x, 2 * (L / gridDim.x), blockIdx.z * 128, B, nt, ntl, nullptr, Cf, cld, N,
                          n_occ, n_aux, Xt, Npad);
}

__global__ void cpad_f32_kernel(const double* C, int N, int n_occ, int rows, int cld, float* Cf) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cld) return;
    int r = e / cld, c = e % cld;
    Cf[e] = (r < N && c < n_occ) ? (float)C[(int64_t)r * n_occ + c] : 0.0f;
}

// Which 16 x 16 sub-tiles (i, j) of a wave's 64 x 64 quadrant of a SYRK tile
// the K reduction reads: rows i < IM (the rest lie at or past row N) and, on a
// quadrant centred on the diagonal, only j <= i.  A wave's shape is fixed for
// the whole launch, so each shape gets its own copy of the k-loop and the
// MFMA sequence stays branch-free.
template <bool DIAG, int IM>
struct SyrkShape {
    static constexpr bool diag = DIAG;
    static constexpr int im = IM;
};

// Runs fn(SyrkShape<...>{}) for the shape of the quadrant at rows qm.., cols
// qn.. (wave-uniform values).
template <class F>
__device__ __forceinline__ void syrk_dispatch(int qm, int qn, int N, F&& fn) {
    const int im = qn > qm ? 0 : min(4, max(0, (N - qm + 15) / 16));
    if (im == 0) return fn(SyrkShape<false, 0>{});
    if (qm == qn) {
        if (im == 4) return fn(SyrkShape<true, 4>{});
        if (im == 3) return fn(SyrkShape<true, 3>{});
        if (im == 2) return fn(SyrkShape<true, 2>{});
        return fn(SyrkShape<true, 1>{});
    }
    if (im == 4) return fn(SyrkShape<false, 4>{});
    if (im == 3) return fn(SyrkShape<false, 3>{});
    if (im == 2) return fn(SyrkShape<false, 2>{});
    return fn(SyrkShape<false, 1>{});
}

// FP32 exchange SYRK on the direct-LDS ring: one wave instruction moves two
// 128-float tile rows (lanes 0-31 the first, 32-63 the second); 16 B chunks
// of row r sit at chunk ^ ((r & 3) << 2) so the four k-rows a fragment read
// touches map to disjoint banks.  FP32 accumulation within a split, partial
// tiles written in FP64 and summed across splits in FP64.
template <int S>
__device__ __forceinline__ void syrk_body_f32(int z, int t, const float* __restrict__ X, int N, int Npad,
                                              int64_t rows_pad, int64_t chunk, double* __restrict__ part) {
    __shared__ float As[S][16 * 128];
    __shared__ float Bs[S][16 * 128];
    int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    const int tj = t - ti * (ti + 1) / 2;
    const int m0 = ti * 128, n0 = tj * 128;
    const int64_t r0 = (int64_t)z * chunk;
    const int64_t r1 = min(rows_pad, r0 + chunk);
    const int nsteps = (int)((r1 - r0) / 16);
    const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    // wave w moves row pairs 2w and 2w+1 (rows 4w .. 4w+3) of A and of B
    auto issue = [&](int step, int buf) {
        int64_t rb = r0 + (int64_t)step * 16;
        if (rb >= rows_pad) rb = rows_pad;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int row = 4 * wave + 2 * q + (lane >> 5);
            const int c = (lane & 31) ^ ((row & 3) << 2);
            const float* ga = X + (rb + row) * Npad + m0 + 4 * c;
            const float* gb = X + (rb + row) * Npad + n0 + 4 * c;
            const int lds_row = 4 * wave + 2 * q;
            __builtin_amdgcn_global_load_lds((const void*)ga, (lds_void_t)(&As[buf][lds_row * 128]), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void*)gb, (lds_void_t)(&Bs[buf][lds_row * 128]), 16, 0, 0);
        }
    };
    f4_t acc[4][4];
    d4_t acc64[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
            acc64[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll
    for (int s = 0; s < S - 1; ++s) issue(s, s);
    syrk_dispatch(m0 + wm, n0 + wn, N, [&](auto shape) {
        constexpr bool DIAG = decltype(shape)::diag;
        constexpr int IM = decltype(shape)::im;
        for (int k = 0; k < nsteps; ++k) {
            if ((k & 3) == 0 && k > 0) {   // FP32 over 64 rows, FP64 across
#pragma unroll
                for (int i = 0; i < IM; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            acc64[i][j][r] += (double)acc[i][j][r];
                            acc[i][j][r] = 0.0f;
                        }
            }
            __builtin_amdgcn_s_waitcnt(((S - 2) * 4 & 0xF) | ((((S - 2) * 4) >> 4) << 14) | (0x7 << 4) | (0xF << 8));
            __builtin_amdgcn_s_barrier();
            issue(k + S - 1, (k + S - 1) % S);
            const float* as = As[k % S];
            const float* bs = Bs[k % S];
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                const int row = kk + lk, sw = (row & 3) << 2;
                float a[4], b[4];
#pragma unroll
                for (int i = 0; i < IM; ++i) {
                    const int m = wm + 16 * i + li;
                    a[i] = as[row * 128 + 4 * ((m >> 2) ^ sw) + (m & 3)];
                }
#pragma unroll
                for (int j = 0; j < (DIAG ? IM : 4); ++j) {
                    const int n = wn + 16 * j + li;
                    b[j] = bs[row * 128 + 4 * ((n >> 2) ^ sw) + (n & 3)];
                }
#pragma unroll
                for (int i = 0; i < IM; ++i)
#pragma unroll
                    for (int j = 0; j < (DIAG ? i + 1 : 4); ++j) acc[i][j] = mfma_f32(a[i], b[j], acc[i][j]);
            }
            __builtin_amdgcn_s_waitcnt(0xC07F);
        }
    });
    __builtin_amdgcn_s_waitcnt(0);
    double* out = part + (int64_t)z * Npad * Npad;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(int64_t)(m0 + wm + 16 * i + 4 * lk + r) * Npad + n0 + wn + 16 * j + li] =
                    acc64[i][j][r] + (double)acc[i][j][r];
}

template <int S>
__global__ __launch_bounds__(256, 2) void syrk_lds_f32_kernel(const float* __restrict__ X, int N, int Npad,
                                                              int64_t rows_pad, int64_t chunk, int ntile,
                                                              double* __restrict__ part) {
    const int nlow = ntile * (ntile + 1) / 2;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    syrk_body_f32<S>(L / nlow, L % nlow, X, N, Npad, rows_pad, chunk, part);
}

// Exchange SYRK, K_part[z] = sum over rows r of split z of Xt[r][m] Xt[r][n],
// for the lower 128 x 128 tiles only.  Rows of Xt are streamed through an
// S-stage LDS ring filled by direct global->LDS loads (global_load_lds, 16 B
// per lane: one wave moves one 1 KB tile row per instruction), so several
// k-steps of loads are in flight without staging registers.  One barrier per
// k-step.  Row r is (P, i) flattened; the buffer carries >= 16 zero rows past
// the last real row, so split ends and the pipeline's look-ahead loads stay
// in bounds and contribute nothing.

template <int S>
__device__ __forceinline__ void syrk_body_f64(int z, int t, const double* __restrict__ X, int N, int Npad,
                                              int64_t rows_pad, int64_t chunk, double* __restrict__ part) {
    constexpr int LDR = 128 + 16;                  // LDS row stride (doubles)
    __shared__ double As[S][16 * LDR];
    __shared__ double Bs[S][16 * LDR];
    int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    const int tj = t - ti * (ti + 1) / 2;
    const int m0 = ti * 128, n0 = tj * 128;
    const int64_t r0 = (int64_t)z * chunk;
    const int64_t r1 = min(rows_pad, r0 + chunk);
    const int nsteps = (int)((r1 - r0) / 16);
    const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    // each wave moves rows 4*wave .. 4*wave+3 of the A and B 16-row slabs.
    // A split's rows plus one 16-row look-ahead (the next split's rows or the
    // zero rows) are reached through buffer resources when their extent fits
    // a 32-bit offset: lane offsets fixed, the step offset a scalar.
    const bool bufok = (r1 - r0 + 16) * Npad * 8 <= INT32_MAX;
#if defined(__HIP_DEVICE_COMPILE__)
    const int nrec = bufok ? (int)((r1 - r0 + 16) * Npad * 8) : 0;
    const __amdgpu_buffer_rsrc_t rsa =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X + r0 * Npad + m0), (short)0, nrec, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsb =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X + r0 * Npad + n0), (short)0, nrec, 0x00020000);
    const int vrow = ((4 * wave) * Npad + 2 * lane) * 8;
    const int last = (int)(r1 - r0);
#endif
    auto issue = [&](int step, int buf) {
        if (bufok) {
#if defined(__HIP_DEVICE_COMPILE__)
            const int so = min(step * 16, last) * Npad * 8;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 4 * wave + q;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rsa, (lds_void_t)(&As[buf][row * LDR]), 16, vrow + q * Npad * 8,
                                                         so, 0, 0);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rsb, (lds_void_t)(&Bs[buf][row * LDR]), 16, vrow + q * Npad * 8,
                                                         so, 0, 0);
            }
#endif
            return;
        }
        int64_t rb = r0 + (int64_t)step * 16;
        if (rb >= rows_pad) rb = rows_pad;          // zero tail rows
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 4 * wave + q;
            const double* ga = X + (rb + row) * Npad + m0 + 2 * lane;
            const double* gb = X + (rb + row) * Npad + n0 + 2 * lane;
            __builtin_amdgcn_global_load_lds((const void*)ga, (lds_void_t)(&As[buf][row * LDR]), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void*)gb, (lds_void_t)(&Bs[buf][row * LDR]), 16, 0, 0);
        }
    };
    d4_t acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < S - 1; ++s) issue(s, s);
    // sub-tiles the reduction never reads are skipped (the upper quadrant of
    // a diagonal tile: its wave only moves data)
    syrk_dispatch(m0 + wm, n0 + wn, N, [&](auto shape) {
        constexpr bool DIAG = decltype(shape)::diag;
        constexpr int IM = decltype(shape)::im;
        for (int k = 0; k < nsteps; ++k) {
            // this wave's loads for step k are done once at most (S-2)*8 younger ones remain
            __builtin_amdgcn_s_waitcnt(((S - 2) * 8 & 0xF) | ((((S - 2) * 8) >> 4) << 14) | (0x7 << 4) | (0xF << 8));
            __builtin_amdgcn_s_barrier();
            issue(k + S - 1, (k + S - 1) % S);
            const double* as = As[k % S];
            const double* bs = Bs[k % S];
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
                double a[4], b[4];
#pragma unroll
                for (int i = 0; i < IM; ++i) a[i] = as[(kk + lk) * LDR + wm + 16 * i + li];
#pragma unroll
                for (int j = 0; j < (DIAG ? IM : 4); ++j) b[j] = bs[(kk + lk) * LDR + wn + 16 * j + li];
#pragma unroll
                for (int i = 0; i < IM; ++i)
#pragma unroll
                    for (int j = 0; j < (DIAG ? i + 1 : 4); ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
            }
            __builtin_amdgcn_s_waitcnt(0xC07F);    // lgkmcnt(0): LDS reads of this buffer done
        }
    });
    __builtin_amdgcn_s_waitcnt(0);
    double* out = part + (int64_t)z * Npad * Npad;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(int64_t)(m0 + wm + 16 * i + 4 * r + lk) * Npad + n0 + wn + 16 * j + li] = acc[i][j][r];
}

template <int S>
__global__ __launch_bounds__(256, 2) void syrk_lds_kernel(const double* __restrict__ X, int N, int Npad,
                                                          int64_t rows_pad, int64_t chunk, int ntile,
                                                          double* __restrict__ part) {
    const int nlow = ntile * (ntile + 1) / 2;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    syrk_body_f64<S>(L / nlow, L % nlow, X, N, Npad, rows_pad, chunk, part);
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

// pair weights of a density matrix: D_mu_mu on the diagonal, D_mu_nu + D_nu_mu off it
__global__ void dpair_density_kernel(const int32_t* pairs, int64_t n_pairs, const double* D, int N, double* dp) {
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    const int mu = pairs[2 * q], nu = pairs[2 * q + 1];
    dp[q] = mu == nu ? D[(int64_t)mu * N + mu] : D[(int64_t)mu * N + nu] + D[(int64_t)nu * N + mu];
}

// gamma_P, one block per auxiliary index at a time (grid-stride, so a small
// grid can run beside the exchange kernels); the sum order per P does not
// depend on the grid.
__global__ __launch_bounds__(256) void gamma_kernel(const double* Bc, int n_aux, int64_t n_pairs, const double* dp,
                                                    double* gamma) {
    __shared__ double sh[4];
    for (int P = blockIdx.x; P < n_aux; P += gridDim.x) {
        const double* row = Bc + (int64_t)P * n_pairs;
        double s = 0.0;
        for (int64_t q = threadIdx.x; q < n_pairs; q += 256) s += row[q] * dp[q];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) gamma[P] = sh[0] + sh[1] + sh[2] + sh[3];
        __syncthreads();
    }
}

// J partials over `per` auxiliary indices per split: item (pair block, split),
// grid-stride over the pb * n_split items.
__global__ __launch_bounds__(256) void jpair_kernel(const double* Bc, int64_t n_pairs, int n_aux, const double* gamma,
                                                    int per, int64_t pb, int n_split, double* jpart) {
    for (int64_t it = blockIdx.x; it < pb * n_split; it += gridDim.x) {
        const int64_t q = (it % pb) * 256 + threadIdx.x;
        const int z = (int)(it / pb);
        if (q >= n_pairs) continue;
        const int p0 = z * per, p1 = min(n_aux, p0 + per);
        double s = 0.0;
        for (int P = p0; P < p1; ++P) s += Bc[(int64_t)P * n_pairs + q] * gamma[P];
        jpart[(int64_t)z * n_pairs + q] = s;
    }
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
    dim3 grid((unsigned)n_tiles(N), (n_aux + PACK_PB - 1) / PACK_PB);
    if (prec == RI_FP64)
        pack_kernel<double><<<grid, 256, 0, st>>>(Bc, n_pairs, map, N, n_tiles(N), n_aux, (double*)B);
    else if (prec == RI_FP32)
        pack_kernel<float><<<grid, 256, 0, st>>>(Bc, n_pairs, map, N, n_tiles(N), n_aux, (float*)B);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

int cpad_ld(int n_occ) { return (n_occ + 127) / 128 * 128; }
int64_t cpad_elems(int N, int n_occ) { return (int64_t)n_tiles_1d(N) * 64 * cpad_ld(n_occ); }


// The FP64 X launch for shape code 4 * (16-row tiles) + (4-row quads); B
// stored as TB (double, or float widened on load).
template <typename TB>
hipError_t x_f64_launch(const TB* b, dim3 grid, int shape, int nt, int64_t ntl, const double* Cp, int cld, int N,
                        int n_occ, int n_aux, double* x, int Npad, hipStream_t st) {
    switch (shape) {
#define XCASE(f, q) case f * 4 + q: x2_kernel_f64<f, q, TB><<<grid, 256, 0, st>>>(b, nt, ntl, Cp, cld, N, n_occ, n_aux, x, Npad); break;
#define XROW(f) XCASE(f, 1) XCASE(f, 2) XCASE(f, 3)
        XROW(0) XROW(1) XROW(2) XROW(3) XROW(4) XROW(5) XROW(6) XROW(7)
        XCASE(1, 0) XCASE(2, 0) XCASE(3, 0) XCASE(4, 0) XCASE(5, 0) XCASE(6, 0) XCASE(7, 0) XCASE(8, 0)
#undef XROW
#undef XCASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t x_transform(const void* B, int prec, int N, int n_aux, int n_occ, const double* C, double* Cp, void* Xt,
                       hipStream_t st) {
    const int nt = n_tiles_1d(N), Npad = xt_ld(N);
    const int mt = (min(n_occ, 128) + 15) / 16;
    dim3 grid(nt, (n_aux + 1) / 2, (n_occ + 127) / 128);
    if (prec == RI_FP32) {
        const float* b = (const float*)B;
        float* x = (float*)Xt;
        const int64_t ntl = n_tiles(N);
        const int cld = cpad_ld(n_occ), rows = nt * 64;
        if (ntl * 4096 * 4 > INT32_MAX || (int64_t)rows * cld * 4 > INT32_MAX) return hipErrorInvalidValue;
        float* Cf = (float*)Cp;      // the C workspace holds twice as many floats as the padded FP64 copy
        cpad_f32_kernel<<<(unsigned)(((int64_t)rows * cld + 255) / 256), 256, 0, st>>>(C, N, n_occ, rows, cld, Cf);
        RI_TRY(hipGetLastError());
        switch (mt) {
#define XCASE(k) case k: x2_kernel_f32<k><<<grid, 256, 0, st>>>(b, nt, ntl, Cf, cld, N, n_occ, n_aux, x, Npad); break;
            XCASE(1) XCASE(2) XCASE(3) XCASE(4) XCASE(5) XCASE(6) XCASE(7) XCASE(8)
#undef XCASE
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (prec != RI_FP64 && prec != X_F64_B32) return hipErrorInvalidValue;
    double* x = (double*)Xt;
    const int64_t ntl = n_tiles(N);
    // occupied rows of one 128-wide chunk: whole 16-row tiles plus, when the
    // last tile would hold 12 rows or fewer, 4-row quads in its place
    int mf = mt, tq = 0;
    if (n_occ <= 128) {
        const int rem = n_occ - 16 * (mt - 1);
        if (rem <= 12) { mf = mt - 1; tq = (rem + 3) / 4; }
    }
    const int cld = cpad_ld(n_occ), rows = nt * 64;
    // buffer-resource offsets are 32-bit: one auxiliary index's packed tiles
    // and the padded C must each stay under 2 GiB (N below about 22,000)
    if (ntl * 4096 * 8 > INT32_MAX || (int64_t)rows * cld * 8 > INT32_MAX) return hipErrorInvalidValue;
    cpad_kernel<<<(unsigned)(((int64_t)rows * cld + 255) / 256), 256, 0, st>>>(C, N, n_occ, rows, cld, Cp);
    RI_TRY(hipGetLastError());
    if (prec == X_F64_B32) return x_f64_launch((const float*)B, grid, mf * 4 + tq, nt, ntl, Cp, cld, N, n_occ, n_aux, x, Npad, st);
    return x_f64_launch((const double*)B, grid, mf * 4 + tq, nt, ntl, Cp, cld, N, n_occ, n_aux, x, Npad, st);
}

int k_split_count(int N, int n_aux, int n_occ) {
    // One round of workgroups: 2 resident 128 x 128 tiles per CU on 256 CUs.
    const int nt = n_tiles_1d(N);
    const int t128 = (nt + 1) / 2;
    const int64_t tiles = (int64_t)t128 * (t128 + 1) / 2;     // lower 128 x 128 tiles
    const int64_t steps = ((int64_t)n_aux * n_occ + 15) / 16;
    int s = (int)std::max<int64_t>(1, 512 / tiles);
    if (s > 64) s = 64;
    if (steps < s) s = (int)std::max<int64_t>(1, steps);
    return s;
}

// Rows of the Xt buffer: n_aux * n_occ rounded up to 16, plus 16 zero rows.
int64_t xt_rows(int n_aux, int n_occ) { return ((int64_t)n_aux * n_occ + 15) / 16 * 16 + 16; }

// Row stride of Xt and of the K partial tiles: N rounded up to 128.
int xt_ld(int N) { return (N + 127) / 128 * 128; }

hipError_t k_syrk(const void* Xt, int prec, int N, int n_aux, int n_occ, double* part, int n_split,
                  double* K, hipStream_t st) {
    if (prec != RI_FP64 && prec != RI_FP32) return hipErrorInvalidValue;
    const int Npad = xt_ld(N), t128 = Npad / 128;
    const int64_t rows = (int64_t)n_aux * n_occ;
    const int64_t rows_pad = (rows + 15) / 16 * 16;
    const int64_t chunk = ((rows_pad + n_split - 1) / n_split + 15) / 16 * 16;
    const int used = (int)((rows_pad + chunk - 1) / chunk);
    const int nlow = t128 * (t128 + 1) / 2;
    if (prec == RI_FP64) {
        double* x = (double*)Xt;
        // zero the padding rows (real rows .. rows_pad + 16)
        RI_TRY(fill(x + rows * Npad, 0.0, (rows_pad + 16 - rows) * Npad, st));
        syrk_lds_kernel<2><<<nlow * used, 256, 0, st>>>(x, N, Npad, rows_pad, chunk, t128, part);
    } else {
        float* x = (float*)Xt;
        // zero padding rows (the region is 512 B aligned: fill it as doubles)
        RI_TRY(fill((double*)(x + rows * Npad), 0.0, (rows_pad + 16 - rows) * Npad / 2, st));
        syrk_lds_f32_kernel<4><<<nlow * used, 256, 0, st>>>(x, N, Npad, rows_pad, chunk, t128, part);
    }
    RI_TRY(hipGetLastError());
    dim3 grid((N + 255) / 256, N);
    kreduce_kernel<<<grid, 256, 0, st>>>(part, used, Npad, N, K);
    return hipGetLastError();
}

int j_split_count(int n_aux) { return n_aux >= 512 ? 16 : 1; }

hipError_t gamma_j(const double* Bc, const int32_t* pairs, int64_t n_pairs, int N, int n_aux, int n_occ,
                   const double* C, double* dpair, double* gamma, double* jpart, int n_jsplit, double* J,
                   hipStream_t st, int cap) {
    if (n_pairs > 0) {
        dpair_kernel<<<(unsigned)((n_pairs + 255) / 256), 256, 0, st>>>(pairs, n_pairs, C, n_occ, dpair);
        RI_TRY(hipGetLastError());
    }
    return gamma_j_pairs(Bc, pairs, n_pairs, N, n_aux, dpair, gamma, jpart, n_jsplit, J, st, cap);
}

hipError_t dpair_density(const int32_t* pairs, int64_t n_pairs, const double* D, int N, double* dpair, hipStream_t st) {
    if (n_pairs == 0) return hipSuccess;
    dpair_density_kernel<<<(unsigned)((n_pairs + 255) / 256), 256, 0, st>>>(pairs, n_pairs, D, N, dpair);
    return hipGetLastError();
}

hipError_t gamma_j_pairs(const double* Bc, const int32_t* pairs, int64_t n_pairs, int N, int n_aux,
                         const double* dpair, double* gamma, double* jpart, int n_jsplit, double* J, hipStream_t st,
                         int cap) {
    RI_TRY(fill(J, 0.0, (int64_t)N * N, st));
    if (n_pairs == 0) return fill(gamma, 0.0, n_aux, st);
    const unsigned pb = (unsigned)((n_pairs + 255) / 256);
    const int64_t items = (int64_t)pb * n_jsplit;
    gamma_kernel<<<cap > 0 ? std::min(n_aux, cap) : n_aux, 256, 0, st>>>(Bc, n_aux, n_pairs, dpair, gamma);
    RI_TRY(hipGetLastError());
    const int per = (n_aux + n_jsplit - 1) / n_jsplit;
    jpair_kernel<<<(unsigned)(cap > 0 ? std::min<int64_t>(items, cap) : items), 256, 0, st>>>(
        Bc, n_pairs, n_aux, gamma, per, pb, n_jsplit, jpart);
    RI_TRY(hipGetLastError());
    jscatter_kernel<<<pb, 256, 0, st>>>(jpart, n_jsplit, pairs, n_pairs, N, J);
    return hipGetLastError();
}

}  // namespace ri

// ------------------------------------------------------------ batched forms
namespace {

// xs = 4 MF + TQ: FP64 takes MF whole tiles and TQ quads, FP32 (TQ = 0) MF
// whole tiles, both from the padded Cq ([64 nt][64], buffer loads).
template <int MF, int TQ, int PREC>
__global__ __launch_bounds__(256, 2) void x_b_kernel(const ri::MolDesc* d, const int* prefix, int n_mol) {
    int mol, loc;
    ri::decode_item(prefix, n_mol, blockIdx.x, mol, loc);
    const ri::MolDesc& m = d[mol];
    if (!m.state[0] || m.xs != 4 * MF + TQ) return;
    const int I = loc % m.nt, P0 = 2 * (loc / m.nt);
    if constexpr (PREC == RI_FP64)
        x2_body_f64<MF, TQ, true>(I, P0, 0, (const double*)m.B, m.nt, m.ntl, m.Cq, 64, m.N, m.n_occ, m.n_aux,
                                  (double*)m.Xt, m.npad);
    else if constexpr (PREC == ri::X_F64_B32)
        x2_body_f64<MF, TQ, true, float>(I, P0, 0, (const float*)m.B, m.nt, m.ntl, m.Cq, 64, m.N, m.n_occ,
                                         m.n_aux, (double*)m.Xt, m.npad);
    else
        x2_body_f32<MF, true>(I, P0, 0, (const float*)m.B, m.nt, m.ntl, nullptr, (const float*)m.Cq, 64, m.N,
                              m.n_occ, m.n_aux, (float*)m.Xt, m.npad);
}

// one block per 64-row block of each active molecule: Cq = C zero-padded
template <typename T>
__global__ void cpad_b_kernel(const ri::MolDesc* d, const int* prefix, int n_mol) {
    int mol, blk;
    ri::decode_item(prefix, n_mol, blockIdx.x, mol, blk);
    const ri::MolDesc& m = d[mol];
    if (!m.state[0]) return;
    T* q = (T*)m.Cq;
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        const int r = 64 * blk + (e >> 6), c = e & 63;
        q[(int64_t)r * 64 + c] = (T)((r < m.N && c < m.n_occ) ? m.C[(int64_t)r * m.n_occ + c] : 0.0);
    }
}

template <int PREC>
__global__ __launch_bounds__(256, 2) void syrk_b_kernel(const ri::MolDesc* d, const int* prefix, int n_mol) {
    int mol, loc;
    ri::decode_item(prefix, n_mol, blockIdx.x, mol, loc);
    const ri::MolDesc& m = d[mol];
    if (!m.state[0]) return;
    const int t128 = m.npad / 128, nlow = t128 * (t128 + 1) / 2;
    if (PREC == RI_FP64)
        syrk_body_f64<2>(loc / nlow, loc % nlow, (const double*)m.Xt, m.N, m.npad, m.rows_pad, m.chunk, m.part);
    else
        syrk_body_f32<4>(loc / nlow, loc % nlow, (const float*)m.Xt, m.N, m.npad, m.rows_pad, m.chunk, m.part);
}

// one block per row mu of each molecule: K[mu][nu] = K[nu][mu] = sum_z part[z][mu][nu], nu <= mu
__global__ void kreduce_b_kernel(const ri::MolDesc* d, const int* prefix, int n_mol) {
    int mol, mu;
    ri::decode_item(prefix, n_mol, blockIdx.x, mol, mu);
    const ri::MolDesc& m = d[mol];
    if (!m.state[0]) return;
    const int used = (int)((m.rows_pad + m.chunk - 1) / m.chunk);
    for (int nu = threadIdx.x; nu <= mu; nu += blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < used; ++k) s += m.part[((int64_t)k * m.npad + mu) * m.npad + nu];
        m.K[(int64_t)mu * m.N + nu] = s;
        m.K[(int64_t)nu * m.N + mu] = s;
    }
}

// zero the 16-row-aligned tail of each molecule's Xt (rows n_aux*n_occ .. rows_pad + 16)
template <int PREC>
__global__ void zero_tail_b_kernel(const ri::MolDesc* d, const int* prefix, int n_mol) {
    int mol, loc;
    ri::decode_item(prefix, n_mol, blockIdx.x, mol, loc);
    const ri::MolDesc& m = d[mol];
    if (!m.state[0]) return;
    const int64_t r0 = (int64_t)m.n_aux * m.n_occ, n = (m.rows_pad + 16 - r0) * m.npad;
    for (int64_t e = (int64_t)loc * blockDim.x + threadIdx.x; e < n; e += 16ll * blockDim.x) {   // 16 blocks per molecule
        if (PREC == RI_FP64) ((double*)m.Xt)[r0 * m.npad + e] = 0.0;
        else ((float*)m.Xt)[r0 * m.npad + e] = 0.0f;
    }
}

// gamma and J on compressed pairs, batched: dpair per pair, gamma per P,
// J per pair (full P loop), then scatter into the zeroed dense J.
__global__ void dpair_b_kernel(const ri::MolDesc* d, const int* prefix, int n_mol) {
    int mol, loc;
    ri::decode_item(prefix, n_mol, blockIdx.x, mol, loc);
    const ri::MolDesc& m = d[mol];
    int64_t q = (int64_t)loc * blockDim.x + threadIdx.x;
    if (!m.state[0] || q >= m.n_pairs) return;
    int mu = m.pairs[2 * q], nu = m.pairs[2 * q + 1];
    const double* a = m.C + (int64_t)mu * m.n_occ;
    const double* b = m.C + (int64_t)nu * m.n_occ;
    double s = 0.0;
    for (int i = 0; i < m.n_occ; ++i) s += a[i] * b[i];
    m.dpair[q] = (mu == nu ? 2.0 : 4.0) * s;
}

__global__ __launch_bounds__(256) void gamma_b_kernel(const ri::MolDesc* d, const int* prefix, int n_mol) {
    int mol, P;
    ri::decode_item(prefix, n_mol, blockIdx.x, mol, P);
    const ri::MolDesc& m = d[mol];
    if (!m.state[0]) return;
    const double* row = m.Bc + (int64_t)P * m.n_pairs;
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < m.n_pairs; q += 256) s += row[q] * m.dpair[q];
    __shared__ double sh[4];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) m.gamma[P] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void jfill_b_kernel(const ri::MolDesc* d, const int* prefix, int n_mol) {
    int mol, loc;
    ri::decode_item(prefix, n_mol, blockIdx.x, mol, loc);
    const ri::MolDesc& m = d[mol];
    int64_t e = (int64_t)loc * blockDim.x + threadIdx.x;
    if (!m.state[0] || e >= (int64_t)m.N * m.N) return;
    m.J[e] = 0.0;
}

__global__ void jpair_b_kernel(const ri::MolDesc* d, const int* prefix, int n_mol) {
    int mol, loc;
    ri::decode_item(prefix, n_mol, blockIdx.x, mol, loc);
    const ri::MolDesc& m = d[mol];
    int64_t q = (int64_t)loc * blockDim.x + threadIdx.x;
    if (!m.state[0] || q >= m.n_pairs) return;
    double s = 0.0;
    for (int P = 0; P < m.n_aux; ++P) s += m.Bc[(int64_t)P * m.n_pairs + q] * m.gamma[P];
    int mu = m.pairs[2 * q], nu = m.pairs[2 * q + 1];
    m.J[(int64_t)mu * m.N + nu] = s;
    m.J[(int64_t)nu * m.N + mu] = s;
}

}  // namespace

namespace ri {

hipError_t x_transform_b(const MolDesc* d, const int* prefix, int n_mol, int total, int xs, int prec, hipStream_t st) {
    if (total <= 0) return hipSuccess;
    if (prec == RI_FP64) {
        switch (xs) {
#define XB(f, q) case 4 * f + q: x_b_kernel<f, q, RI_FP64><<<total, 256, 0, st>>>(d, prefix, n_mol); break;
            XB(0, 1) XB(0, 2) XB(0, 3) XB(1, 0) XB(1, 1) XB(1, 2) XB(1, 3) XB(2, 0)
            XB(2, 1) XB(2, 2) XB(2, 3) XB(3, 0) XB(3, 1) XB(3, 2) XB(3, 3) XB(4, 0)
#undef XB
            default: return hipErrorInvalidValue;
        }
    } else if (prec == X_F64_B32) {
        switch (xs) {
#define XB(f, q) case 4 * f + q: x_b_kernel<f, q, X_F64_B32><<<total, 256, 0, st>>>(d, prefix, n_mol); break;
            XB(0, 1) XB(0, 2) XB(0, 3) XB(1, 0) XB(1, 1) XB(1, 2) XB(1, 3) XB(2, 0)
            XB(2, 1) XB(2, 2) XB(2, 3) XB(3, 0) XB(3, 1) XB(3, 2) XB(3, 3) XB(4, 0)
#undef XB
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (xs) {
#define XB(f) case 4 * f: x_b_kernel<f, 0, RI_FP32><<<total, 256, 0, st>>>(d, prefix, n_mol); break;
            XB(1) XB(2) XB(3) XB(4)
#undef XB
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t cpad_b(const MolDesc* d, const int* prefix, int n_mol, int total, int prec, hipStream_t st) {
    if (total <= 0) return hipSuccess;
    if (prec == RI_FP64) cpad_b_kernel<double><<<total, 256, 0, st>>>(d, prefix, n_mol);
    else cpad_b_kernel<float><<<total, 256, 0, st>>>(d, prefix, n_mol);
    return hipGetLastError();
}

hipError_t syrk_b(const MolDesc* d, const int* prefix, int n_mol, int total, int prec, hipStream_t st) {
    if (total <= 0) return hipSuccess;
    if (prec == RI_FP64) syrk_b_kernel<RI_FP64><<<total, 256, 0, st>>>(d, prefix, n_mol);
    else syrk_b_kernel<RI_FP32><<<total, 256, 0, st>>>(d, prefix, n_mol);
    return hipGetLastError();
}

hipError_t kreduce_b(const MolDesc* d, const int* prefix, int n_mol, int total, hipStream_t st) {
    if (total <= 0) return hipSuccess;
    kreduce_b_kernel<<<total, 256, 0, st>>>(d, prefix, n_mol);
    return hipGetLastError();
}

hipError_t zero_tail_b(const MolDesc* d, const int* prefix, int n_mol, int total, int prec, hipStream_t st) {
    if (total <= 0) return hipSuccess;
    if (prec == RI_FP64) zero_tail_b_kernel<RI_FP64><<<total, 256, 0, st>>>(d, prefix, n_mol);
    else zero_tail_b_kernel<RI_FP32><<<total, 256, 0, st>>>(d, prefix, n_mol);
    return hipGetLastError();
}

hipError_t gamma_j_b(const MolDesc* d, int n_mol, const int* pre_pairs, int tot_pairs, const int* pre_aux, int tot_aux,
                     const int* pre_n2, int tot_n2, hipStream_t st) {
    if (tot_n2 > 0) jfill_b_kernel<<<tot_n2, 256, 0, st>>>(d, pre_n2, n_mol);
    if (tot_pairs > 0) dpair_b_kernel<<<tot_pairs, 256, 0, st>>>(d, pre_pairs, n_mol);
    if (tot_aux > 0) gamma_b_kernel<<<tot_aux, 256, 0, st>>>(d, pre_aux, n_mol);
    if (tot_pairs > 0) jpair_b_kernel<<<tot_pairs, 256, 0, st>>>(d, pre_pairs, n_mol);
    return hipGetLastError();
}

}  // namespace ri
