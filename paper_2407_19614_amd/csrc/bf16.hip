// Split-BF16 exchange contractions (precision extension).  A value v is held
// as NS bfloat16 parts v = h + m (+ l): h = bf16(v), m = bf16(v - h),
// l = bf16(v - h - m).  A product uses every pair of parts whose orders add
// to at most NS - 1 (NS = 2: 3 products, NS = 3: 6 products) on
// v_mfma_f32_16x16x32_bf16, accumulated in FP32 within a 64-deep chunk and in
// FP64 across chunks.
//
// Layouts:
//   B  [NS][n_aux][nt][nt][64][64]  full square tiles: tile (I,J) holds
//      B^P[64I + r][64J + c] at r*64 + c (both triangles stored, so a row
//      block is contiguous along nu in every tile).
//   Ct [NS][W][Npad]   C_occ^T parts, W = 16 * MT occupied rows (zero padded).
//   Xb [NS][Npad][R]   X parts with mu as the row and (P, i) -> P*n_occ + i
//      as the contiguous K index, R = n_aux*n_occ rounded up to 64.
// MFMA operand layout (16x16x32 bf16): lane l supplies row l%16 and
// k = 8*(l/16) + 0..7 of A, column l%16 and the same k of B, and receives
// D[4*(l/16) + r][l%16].
#include "kernels.h"

namespace {

typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split_parts(double v, int ns, __bf16* out) {
    __bf16 h = (__bf16)(float)v;
    double r = v - (double)(float)h;
    out[0] = h;
    __bf16 m = (__bf16)(float)r;
    out[1] = m;
    if (ns > 2) out[2] = (__bf16)(float)(r - (double)(float)m);
}

// B parts from the compressed tensor: one block per (tile (I,J), P)
template <int NS>
__global__ __launch_bounds__(256) void pack_bf16_kernel(const double* Bc, int64_t n_pairs, const int32_t* map,
                                                        int N, int nt, int n_aux, __bf16* B) {
    const int t = blockIdx.x, P = blockIdx.y;
    const int I = t / nt, J = t % nt;
    const double* row = Bc + (int64_t)P * n_pairs;
    const int64_t plane = (int64_t)n_aux * nt * nt * 4096;
    __bf16* out = B + ((int64_t)P * nt * nt + t) * 4096;
    for (int e = threadIdx.x; e < 4096; e += 256) {
        int mu = 64 * I + (e >> 6), nu = 64 * J + (e & 63);
        double v = 0.0;
        if (mu < N && nu < N) {
            int a = max(mu, nu), b = min(mu, nu);
            int32_t q = map[(int64_t)a * N + b];
            if (q >= 0) v = row[q];
        }
        __bf16 p[3];
        split_parts(v, NS, p);
#pragma unroll
        for (int k = 0; k < NS; ++k) out[k * plane + e] = p[k];
    }
}

// Ct parts: Ct[k][i][nu] = part k of C[nu][i]
template <int NS>
__global__ void csplit_kernel(const double* C, int N, int n_occ, int W, int Npad, __bf16* Ct) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)W * Npad) return;
    int i = e / Npad, nu = e % Npad;
    double v = (i < n_occ && nu < N) ? C[(int64_t)nu * n_occ + i] : 0.0;
    __bf16 p[3];
    split_parts(v, NS, p);
    const int64_t plane = (int64_t)W * Npad;
#pragma unroll
    for (int k = 0; k < NS; ++k) Ct[k * plane + e] = p[k];
}

// zero Xb rows mu >= 64*nt and columns >= n_aux*n_occ (never written by the X kernel)
__global__ void xb_pad_kernel(__bf16* Xb, int ns, int Npad, int64_t R, int rows_written, int64_t cols_written) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t pad_cols = R - cols_written;
    const int64_t n_a = (int64_t)(Npad - rows_written) * R;        // whole padding rows
    const int64_t n_b = (int64_t)rows_written * pad_cols;          // padding columns of written rows
    const int64_t per = n_a + n_b;
    if (e >= per * ns) return;
    const int k = e / per;
    int64_t f = e % per, idx;
    if (f < n_a) idx = (int64_t)rows_written * R + f;
    else {
        f -= n_a;
        idx = (f / pad_cols) * R + cols_written + f % pad_cols;
    }
    Xb[(int64_t)k * Npad * R + idx] = (__bf16)0.0f;
}

// Both contractions stream their operands through a three-stage LDS ring
// filled by direct global->LDS loads (16 B per lane; one wave instruction
// moves 16 rows x 64 B, i.e. a 32-deep k-slice of 16 rows).  Each 64 B row
// holds four 16 B chunks; chunk c of row r sits at c ^ ((r >> 2) & 3) so that
// the 16 rows one fragment read touches fall on distinct banks.  A stage is
// consumed two iterations after it is issued (one barrier per stage).
//
// Accumulation: the leading product (part 0 x part 0) of every 32-deep MFMA
// starts from zero and is added to an FP64 accumulator at once; the
// correction products (orders 1 and 2, at most 2^-8 of the leading term)
// share an FP32 accumulator.  Rounding therefore costs one FP32 rounding of a
// 32-term partial sum per fold instead of a chain of them.
constexpr int RING = 3;
constexpr int ROWB = 32;   // bf16 per ring row (one 32-deep k-slice)

__device__ __forceinline__ int swz(int row, int chunk) { return chunk ^ ((row >> 2) & 3); }

// s_waitcnt with vmcnt = n (expcnt / lgkmcnt not waited on)
template <int n>
__device__ __forceinline__ void wait_vm() {
    static_assert(n >= 0 && n < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

__device__ __forceinline__ bf8_t lds_frag(const __bf16* base, int row, int lk) {
    return *(const bf8_t*)(base + row * ROWB + 8 * swz(row, lk));
}

// X for items (row block I2 of 128 rows, auxiliary P), item = I2 + nt2 * P,
// items b, b + G, ... for block b of G (persistent).  D[mu][i] = sum_nu
// B^P[mu][nu] C[nu][i]; wave w owns mu rows 32w .. 32w+31 of the block and
// all MT occupied tiles.
template <int NS, int MT>
__global__ __launch_bounds__(256, 1) void x_bf16_kernel(const __bf16* __restrict__ B, int nt, int n_aux,
                                                        const __bf16* __restrict__ Ct, int Npad, int n_occ,
                                                        __bf16* __restrict__ Xb, int64_t R) {
    constexpr int W = 16 * MT;
    constexpr int SB = NS * 128 * ROWB, SC = NS * W * ROWB, STAGE = SB + SC;
    constexpr int NB = NS * 8 / 4;                 // B instructions per wave per stage
    constexpr int NCI = NS * MT, NC = (NCI + 3) / 4;   // C instructions (total, per wave)
    constexpr int LOADS = NB + NC;
    __shared__ __attribute__((aligned(16))) __bf16 ring[RING * STAGE];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int nt2 = (nt + 1) / 2, spi = 2 * nt;    // stages per item
    const int64_t n_items = (int64_t)nt2 * n_aux;
    const int64_t mine = n_items > blockIdx.x ? (n_items - 1 - blockIdx.x) / gridDim.x + 1 : 0;
    const int64_t total = mine * spi;
    const int64_t bplane = (int64_t)n_aux * nt * nt * 4096;
    const int64_t cplane = (int64_t)W * Npad;
    const int lrow = lane >> 2, lch = lane & 3;    // row within a 16-row load group, chunk

    auto issue = [&](int64_t g) {
        if (g >= total) g = total - 1;             // tail: reload the last stage (never read)
        const int64_t item = blockIdx.x + (g / spi) * gridDim.x;
        const int s = (int)(g % spi), J = s >> 1, ks = s & 1;
        const int I2 = (int)(item % nt2), P = (int)(item / nt2);
        __bf16* st = ring + (int)(g % RING) * STAGE;
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int t = wave + 4 * u, p = t >> 3, rg = t & 7;
            const int row = 16 * rg + lrow;
            const int I = min(2 * I2 + (row >> 6), nt - 1);
            const __bf16* src = B + p * bplane + (((int64_t)P * nt + I) * nt + J) * 4096 + (row & 63) * 64 +
                                32 * ks + 8 * swz(row, lch);
            __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_t)(st + (p * 128 + 16 * rg) * ROWB), 16, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < NC; ++u) {
            const int t = min(wave + 4 * u, NCI - 1), q = t / MT, mg = t % MT;
            const int row = 16 * mg + lrow;
            const __bf16* src = Ct + q * cplane + (int64_t)row * Npad + 64 * J + 32 * ks + 8 * swz(row, lch);
            __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_t)(st + SB + (q * W + 16 * mg) * ROWB), 16,
                                             0, 0);
        }
    };

    d4_t acc64[2][MT];
    f4_t accc[2][MT];
    const f4_t zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int m = 0; m < MT; ++m) { acc64[f][m] = d4_t{0, 0, 0, 0}; accc[f][m] = zero; }
    if (total == 0) return;
    issue(0);
    issue(1);
    for (int64_t g = 0; g < total; ++g) {
        wait_vm<LOADS>();
        __builtin_amdgcn_s_barrier();
        issue(g + 2);
        const __bf16* sb = ring + (int)(g % RING) * STAGE;
        const __bf16* sc = sb + SB;
        bf8_t a[2][NS];
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int p = 0; p < NS; ++p) a[f][p] = lds_frag(sb + p * 128 * ROWB, 32 * wave + 16 * f + li, lk);
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            bf8_t c[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) c[q] = lds_frag(sc + q * W * ROWB, 16 * m + li, lk);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
                const f4_t h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f][0], c[0], zero, 0, 0, 0);
#pragma unroll
                for (int p = 0; p < NS; ++p)
#pragma unroll
                    for (int q = 0; q < NS; ++q)
                        if (p + q > 0 && p + q < NS)
                            accc[f][m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f][p], c[q], accc[f][m], 0, 0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) acc64[f][m][r] += (double)h[r];
            }
        }
        if ((g + 1) % spi == 0) {                  // item complete: write X parts, reset
            const int64_t item = blockIdx.x + (g / spi) * gridDim.x;
            const int I2 = (int)(item % nt2), P = (int)(item / nt2);
            const int64_t xplane = (int64_t)Npad * R;
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int m = 0; m < MT; ++m) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int mu = 128 * I2 + 32 * wave + 16 * f + 4 * lk + r, i = 16 * m + li;
                        if (mu < 64 * nt && i < n_occ) {
                            __bf16 pt[3];
                            split_parts(acc64[f][m][r] + (double)accc[f][m][r], NS, pt);
                            const int64_t o = (int64_t)mu * R + (int64_t)P * n_occ + i;
#pragma unroll
                            for (int k = 0; k < NS; ++k) Xb[k * xplane + o] = pt[k];
                        }
                    }
                    acc64[f][m] = d4_t{0, 0, 0, 0};
                    accc[f][m] = zero;
                }
        }
    }
    wait_vm<0>();
}

// K partials over lower 128 x 128 tiles, split over the K index in multiples
// of 32: part[z][mu][nu] = sum_r X[mu][r] X[nu][r] (split products).  Wave w
// owns the 64 x 64 quarter (w / 2, w % 2).
template <int NS>
__global__ __launch_bounds__(256, 1) void syrk_bf16_kernel(const __bf16* __restrict__ Xb, int Npad, int64_t R,
                                                           int64_t chunk, int ntile, double* __restrict__ part) {
    constexpr int SA = NS * 128 * ROWB, STAGE = 2 * SA;
    constexpr int LOADS = 2 * NS * 8 / 4;
    __shared__ __attribute__((aligned(16))) __bf16 ring[RING * STAGE];
    const int nlow = ntile * (ntile + 1) / 2;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int z = L / nlow, t = L % nlow;
    int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    const int tj = t - ti * (ti + 1) / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int lrow = lane >> 2, lch = lane & 3;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int64_t r0 = (int64_t)z * chunk, r1 = min(R, r0 + chunk);
    const int nst = (int)((r1 - r0) / ROWB);
    const int64_t xplane = (int64_t)Npad * R;

    auto issue = [&](int s) {
        if (s >= nst) s = nst - 1;
        const int64_t rr = r0 + (int64_t)s * ROWB;
        __bf16* st = ring + (s % RING) * STAGE;
#pragma unroll
        for (int u = 0; u < LOADS; ++u) {
            const int tt = wave + 4 * u, side = tt / (NS * 8), rem = tt % (NS * 8), p = rem >> 3, rg = rem & 7;
            const int row = 16 * rg + lrow;
            const int base = side ? tj * 128 : ti * 128;
            const __bf16* src = Xb + p * xplane + (int64_t)(base + row) * R + rr + 8 * swz(row, lch);
            __builtin_amdgcn_global_load_lds((const void*)src, (lds_void_t)(st + side * SA + (p * 128 + 16 * rg) * ROWB),
                                             16, 0, 0);
        }
    };

    d4_t acc64[4][4];
    f4_t accc[4][4];
    const f4_t zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) { acc64[i][j] = d4_t{0, 0, 0, 0}; accc[i][j] = zero; }
    if (nst > 0) {
        issue(0);
        issue(1);
        for (int s = 0; s < nst; ++s) {
            wait_vm<LOADS>();
            __builtin_amdgcn_s_barrier();
            issue(s + 2);
            const __bf16* sa = ring + (s % RING) * STAGE;
            const __bf16* sbb = sa + SA;
            bf8_t a[4][NS], b[4][NS];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int p = 0; p < NS; ++p) {
                    a[i][p] = lds_frag(sa + p * 128 * ROWB, wm + 16 * i + li, lk);
                    b[i][p] = lds_frag(sbb + p * 128 * ROWB, wn + 16 * i + li, lk);
                }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const f4_t h = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][0], b[j][0], zero, 0, 0, 0);
#pragma unroll
                    for (int p = 0; p < NS; ++p)
#pragma unroll
                        for (int q = 0; q < NS; ++q)
                            if (p + q > 0 && p + q < NS)
                                accc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i][p], b[j][q], accc[i][j], 0, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)h[r];
                }
            if ((s & 7) == 7) {                    // corrections: FP32 over 256 rows, FP64 across
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            acc64[i][j][r] += (double)accc[i][j][r];
                            accc[i][j][r] = 0.f;
                        }
            }
        }
        wait_vm<0>();
    }
    double* out = part + (int64_t)z * Npad * Npad;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(int64_t)(ti * 128 + wm + 16 * i + 4 * lk + r) * Npad + tj * 128 + wn + 16 * j + li] =
                    acc64[i][j][r] + (double)accc[i][j][r];
}

__global__ void kreduce_bf_kernel(const double* part, int n_split, int Npad, int N, double* K) {
    int nu = blockIdx.x * blockDim.x + threadIdx.x, mu = blockIdx.y;
    if (nu > mu || mu >= N) return;
    double s = 0.0;
    for (int k = 0; k < n_split; ++k) s += part[((int64_t)k * Npad + mu) * Npad + nu];
    K[(int64_t)mu * N + nu] = s;
    K[(int64_t)nu * N + mu] = s;
}

}  // namespace

namespace ri {

int bf16_parts(int prec) { return prec == RI_BF16X6 ? 3 : 2; }
int64_t bf16_R(int n_aux, int n_occ) { return ((int64_t)n_aux * n_occ + 63) / 64 * 64; }
int64_t bf16_ct_elems(int N, int n_occ) { return (int64_t)((n_occ + 15) / 16) * 16 * xt_ld(N); }
int64_t bf16_xb_elems(int N, int n_aux, int n_occ) { return (int64_t)xt_ld(N) * bf16_R(n_aux, n_occ); }

hipError_t pack_b_bf16(const double* Bc, int64_t n_pairs, const int32_t* map, int N, int n_aux, void* B, int prec,
                       hipStream_t st) {
    const int nt = n_tiles_1d(N);
    dim3 grid(nt * nt, n_aux);
    if (prec == RI_BF16X6) pack_bf16_kernel<3><<<grid, 256, 0, st>>>(Bc, n_pairs, map, N, nt, n_aux, (__bf16*)B);
    else pack_bf16_kernel<2><<<grid, 256, 0, st>>>(Bc, n_pairs, map, N, nt, n_aux, (__bf16*)B);
    return hipGetLastError();
}

int bf16_split_count(int N, int n_aux, int n_occ) {
    // one round of workgroups: one resident 128 x 128 tile per CU (LDS-bound)
    const int t128 = xt_ld(N) / 128;
    const int64_t tiles = (int64_t)t128 * (t128 + 1) / 2;
    const int64_t steps = bf16_R(n_aux, n_occ) / 32;
    int s = (int)std::max<int64_t>(1, device_cus() / tiles);
    if (s > 64) s = 64;
    if (steps < s) s = (int)std::max<int64_t>(1, steps);
    return s;
}

hipError_t x_transform_bf16(const void* B, int prec, int N, int n_aux, int n_occ, const double* C, void* Ct,
                            void* Xb, hipStream_t st) {
    const int ns = bf16_parts(prec), nt = n_tiles_1d(N), Npad = xt_ld(N);
    const int mt = (n_occ + 15) / 16, W = mt * 16;
    if (n_occ > 128) return hipErrorInvalidValue;
    const int64_t R = bf16_R(n_aux, n_occ);
    __bf16* ct = (__bf16*)Ct;
    __bf16* xb = (__bf16*)Xb;
    const int64_t ce = (int64_t)W * Npad;
    if (ns == 3) csplit_kernel<3><<<(unsigned)((ce + 255) / 256), 256, 0, st>>>(C, N, n_occ, W, Npad, ct);
    else csplit_kernel<2><<<(unsigned)((ce + 255) / 256), 256, 0, st>>>(C, N, n_occ, W, Npad, ct);
    RI_TRY(hipGetLastError());
    const int rows_written = nt * 64;
    const int64_t cols = (int64_t)n_aux * n_occ;
    const int64_t padn = ((int64_t)(Npad - rows_written) * R + (int64_t)rows_written * (R - cols)) * ns;
    if (padn > 0) {
        xb_pad_kernel<<<(unsigned)((padn + 255) / 256), 256, 0, st>>>(xb, ns, Npad, R, rows_written, cols);
        RI_TRY(hipGetLastError());
    }
    const int64_t n_items = (int64_t)((nt + 1) / 2) * n_aux;
    const unsigned grid = (unsigned)std::min<int64_t>(n_items, device_cus());
    const __bf16* b = (const __bf16*)B;
#define XB(NS, M) case M: x_bf16_kernel<NS, M><<<grid, 256, 0, st>>>(b, nt, n_aux, ct, Npad, n_occ, xb, R); break;
    if (ns == 3) {
        switch (mt) { XB(3, 1) XB(3, 2) XB(3, 3) XB(3, 4) XB(3, 5) XB(3, 6) XB(3, 7) XB(3, 8) default: return hipErrorInvalidValue; }
    } else {
        switch (mt) { XB(2, 1) XB(2, 2) XB(2, 3) XB(2, 4) XB(2, 5) XB(2, 6) XB(2, 7) XB(2, 8) default: return hipErrorInvalidValue; }
    }
#undef XB
    return hipGetLastError();
}

hipError_t k_syrk_bf16(const void* Xb, int prec, int N, int n_aux, int n_occ, double* part, int n_split, double* K,
                       hipStream_t st) {
    const int ns = bf16_parts(prec), Npad = xt_ld(N);
    const int64_t R = bf16_R(n_aux, n_occ);
    const __bf16* xb = (const __bf16*)Xb;
    const int t128 = Npad / 128, nlow = t128 * (t128 + 1) / 2;
    const int64_t chunk = ((R + n_split - 1) / n_split + 31) / 32 * 32;
    const int used = (int)((R + chunk - 1) / chunk);
    if (ns == 3) syrk_bf16_kernel<3><<<nlow * used, 256, 0, st>>>(xb, Npad, R, chunk, t128, part);
    else syrk_bf16_kernel<2><<<nlow * used, 256, 0, st>>>(xb, Npad, R, chunk, t128, part);
    RI_TRY(hipGetLastError());
    dim3 g2((N + 255) / 256, N);
    kreduce_bf_kernel<<<g2, 256, 0, st>>>(part, used, Npad, N, K);
    return hipGetLastError();
}

}  // namespace ri
