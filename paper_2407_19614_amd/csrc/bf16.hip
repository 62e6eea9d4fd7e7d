// Split-BF16 exchange contractions (precision extension).  A value v is held
// as NS bfloat16 parts v = h + m (+ l): h = bf16(v), m = bf16(v - h),
// l = bf16(v - h - m).  A product uses every pair of parts whose orders add
// to at most NS - 1 (NS = 2: 3 products, NS = 3: 6 products) on
// v_mfma_f32_16x16x32_bf16, accumulated in FP32 within a 64-deep chunk and in
// FP64 across chunks.
//
// Layouts:
//   B  [n_aux][nt][nt][2][NS][64][32]  full square tiles (both triangles):
//      part k of B^P[64I + r][64J + 32h + c] sits in tile (I,J) of P at
//      (h*NS + k)*2048 + r*32 + c, so the 32-deep half h of 16 consecutive
//      rows is one contiguous 1 KB run and the NS parts of a tile half are
//      adjacent.
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
    __bf16* out = B + ((int64_t)P * nt * nt + t) * NS * 4096;
    for (int e = threadIdx.x; e < 4096; e += 256) {
        int mu = 64 * I + ((e >> 5) & 63), nu = 64 * J + 32 * (e >> 11) + (e & 31);
        double v = 0.0;
        if (mu < N && nu < N) {
            int a = max(mu, nu), b = min(mu, nu);
            int32_t q = map[(int64_t)a * N + b];
            if (q >= 0) v = row[q];
        }
        __bf16 p[3];
        split_parts(v, NS, p);
#pragma unroll
        for (int k = 0; k < NS; ++k) out[((e >> 11) * NS + k) * 2048 + (e & 2047)] = p[k];
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

// Both contractions run 8 waves per workgroup (two per SIMD) and stage shared
// operands through a three-slot LDS ring filled by direct global->LDS loads
// (16 B per lane; one wave instruction moves 16 rows x 64 B, a 32-deep
// k-slice of 16 rows).  Each 64 B ring row holds four 16 B chunks; chunk c of
// row r sits at c ^ ((r >> 1) & 3), so any 8 consecutive lanes of a fragment
// read (8 rows, same chunk) touch 8 distinct 16 B bank groups.  A slot is
// consumed two stages after it is issued, with one barrier per stage.
//
// Accumulation per output tile: the leading product (part 0 x part 0) of each
// 32-deep step starts from zero and is added to an FP64 accumulator at once;
// the correction products (orders 1 .. NS-1, at most 2^-8 of the leading
// term) share an FP32 accumulator that is folded into the FP64 one every
// eight steps.  The leading term thus carries one FP32 rounding per 32-term
// partial sum.
constexpr int RING = 3;
constexpr int ROWB = 32;   // bf16 per ring row (one 32-deep k-slice)

__device__ __forceinline__ int swz(int row, int chunk) { return chunk ^ ((row >> 1) & 3); }

// s_waitcnt with vmcnt = n (expcnt / lgkmcnt not waited on)
template <int n>
__device__ __forceinline__ void wait_vm() {
    static_assert(n >= 0 && n < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

__device__ __forceinline__ bf8_t lds_frag(const __bf16* base, int row, int lk) {
    return *(const bf8_t*)(base + row * ROWB + 8 * swz(row, lk));
}

// Buffer resource over `bytes` bytes at `base` (raw buffer, 32-bit offsets).
// Loads go through buffer instructions with the stage-dependent part of the
// address in the scalar offset and a loop-invariant lane offset, so no
// vector register is rewritten between a load's issue and its completion.
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, int64_t bytes) {
    const int n = (int)(bytes < 0x7fffffff ? bytes : 0x7fffffff);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, 0x00020000);
}

// One 32-deep split product: leading term into the FP64 accumulator,
// corrections into the FP32 one (see above).
template <int NS>
__device__ __forceinline__ void split_mfma(const bf8_t (&a)[NS], const bf8_t (&b)[NS], d4_t& acc, f4_t& corr) {
#pragma unroll
    for (int o = 1; o < NS; ++o)
#pragma unroll
        for (int p = 0; p <= o; ++p) corr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[p], b[o - p], corr, 0, 0, 0);
    const f4_t t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], f4_t{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] += (double)t[r];
}

__device__ __forceinline__ void fold(d4_t& acc, f4_t& corr) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        acc[r] += (double)corr[r];
        corr[r] = 0.f;
    }
}

// X for items (row block I2 of 128 rows, auxiliary pair P0 = 2 Pp, P0 + 1),
// item = I2 + nt2 * Pp, items b, b + G, ... for workgroup b of G
// (persistent).  D[mu][i] = sum_nu B^P[mu][nu] C[nu][i].  One ring stage holds the B
// parts of both indices' 128 rows and one C slice, so each C slice serves
// two auxiliary indices (it is about half of a one-index stage: with one
// index per item the same kernel shape took 6.0 ms for BF16X6 at N=1000,
// against 4.8).  Waves 0-3 take index P0 and waves 4-7 index P0 + 1; wave w
// owns rows 32 (w % 4) .. +31 and every occupied column tile.  RING2 slots
// (one or two stages in flight while one is multiplied, as LDS allows).
// Item, stage and slot advance by counters; rows of a tile index >= nt load
// tile nt - 1 and are never written.  With an odd n_aux the last pair's
// second index reloads index n_aux - 1 and is not stored.
template <int NS> struct Bf16PairRing { static constexpr int value = NS == 3 ? 2 : 3; };

template <int NS, int MT>
__global__ __launch_bounds__(512, 1) void x_bf16p_kernel(const __bf16* __restrict__ B, int nt, int n_aux,
                                                         const __bf16* __restrict__ Ct, int Npad, int n_occ,
                                                         __bf16* __restrict__ Xb, int64_t R) {
#if defined(__HIP_DEVICE_COMPILE__)
    constexpr int RING2 = Bf16PairRing<NS>::value;
    constexpr int W = 16 * MT;
    constexpr int SB = 2 * NS * 128 * ROWB, SC = NS * W * ROWB, STAGE = SB + SC;
    constexpr int NB = 2 * NS;                         // B instructions per wave per stage
    constexpr int NCI = NS * MT, NC = (NCI + 7) / 8;   // C instructions (total, per wave)
    constexpr int LOADS = NB + NC;                     // VMEM ops per wave per stage
    __shared__ __attribute__((aligned(16))) __bf16 ring[RING2 * STAGE];
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rg = wave & 3, pi = wave >> 2;
    const int nt2 = (nt + 1) / 2, spi = 2 * nt;        // stages per item
    const int npair = (n_aux + 1) / 2;
    const int n_items = nt2 * npair;
    const int G = gridDim.x;
    const int mine = n_items > (int)blockIdx.x ? (n_items - 1 - (int)blockIdx.x) / G + 1 : 0;
    if (mine == 0) return;
    const int64_t cplane = (int64_t)W * Npad;
    const int lrow = lane >> 2, lch = lane & 3;
    const int bvoff = (lrow * ROWB + 8 * swz(lrow, lch)) * 2;
    const int cvoff = (lrow * Npad + 8 * swz(lrow, lch)) * 2;
    // B instruction u of every wave: index u / NS, part u % NS, 16-row group
    // `wave` of the 128 (tile wave / 4, rows 16 (wave % 4) ..)
    const int bsoff = 16 * (wave & 3) * ROWB * 2;
    const int btl = wave >> 2;
    const __amdgpu_buffer_rsrc_t crs = rsrc(Ct, (int64_t)NS * cplane * 2);
    int csoff[NC], cdst[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) {
        const int t = min(wave + 8 * u, NCI - 1), q = t / MT, mg = t % MT;
        csoff[u] = (int)((q * cplane + (int64_t)16 * mg * Npad) * 2);
        cdst[u] = SB + (q * W + 16 * mg) * ROWB;
    }

    int ij = 0, is = 0, islot = 0;                      // next stage to issue
    int iI2 = (int)blockIdx.x % nt2, iPp = (int)blockIdx.x / nt2;
    auto issue = [&]() {
        const int J = is >> 1, ks = is & 1;
        __bf16* st = ring + islot * STAGE;
        const int I = min(2 * iI2 + btl, nt - 1);
        const int hoff = ks * NS * 2048 * 2;
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int P = min(2 * iPp + x, n_aux - 1);
            const __amdgpu_buffer_rsrc_t brs = rsrc(B + (((int64_t)P * nt + I) * nt + J) * NS * 4096, NS * 4096 * 2);
#pragma unroll
            for (int p = 0; p < NS; ++p)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(brs, (lds_void_t)(st + ((x * NS + p) * 128 + 16 * wave) * ROWB),
                                                         16, bvoff, hoff + p * 2048 * 2 + bsoff, 0, 0);
        }
        const int coff = (64 * J + 32 * ks) * 2;
#pragma unroll
        for (int u = 0; u < NC; ++u)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(crs, (lds_void_t)(st + cdst[u]), 16, cvoff, csoff[u] + coff, 0, 0);
        islot = islot == RING2 - 1 ? 0 : islot + 1;
        if (is + 1 < spi) ++is;
        else if (ij + 1 < mine) {
            is = 0;
            ++ij;
            const int item = (int)blockIdx.x + ij * G;
            iI2 = item % nt2;
            iPp = item / nt2;
        }   // else: stay on the last stage (tail reloads land in a slot that is never read)
    };

    d4_t acc[2][MT];
    f4_t corr[2][MT];
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int m = 0; m < MT; ++m) { acc[f][m] = d4_t{0, 0, 0, 0}; corr[f][m] = f4_t{0.f, 0.f, 0.f, 0.f}; }
    int cj = 0, cs = 0, cslot = 0;
    int cI2 = (int)blockIdx.x % nt2, cPp = (int)blockIdx.x / nt2;
    const int64_t xplane = (int64_t)Npad * R;
#pragma unroll
    for (int r = 0; r < RING2 - 1; ++r) issue();
    while (true) {
        wait_vm<LOADS * (RING2 - 2)>();
        __builtin_amdgcn_s_barrier();
        issue();
        const __bf16* sb = ring + cslot * STAGE;
        const __bf16* sc = sb + SB;
        cslot = cslot == RING2 - 1 ? 0 : cslot + 1;
        bf8_t a[2][NS];
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int p = 0; p < NS; ++p) a[f][p] = lds_frag(sb + (pi * NS + p) * 128 * ROWB, 32 * rg + 16 * f + li, lk);
#pragma unroll
        for (int mi = 0; mi < MT; ++mi) {
            bf8_t c[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) c[q] = lds_frag(sc + q * W * ROWB, 16 * mi + li, lk);
#pragma unroll
            for (int f = 0; f < 2; ++f) split_mfma<NS>(a[f], c, acc[f][mi], corr[f][mi]);
        }
        if ((cs & 7) == 7) {
#pragma unroll
            for (int f = 0; f < 2; ++f)
#pragma unroll
                for (int mi = 0; mi < MT; ++mi) fold(acc[f][mi], corr[f][mi]);
        }
        if (++cs < spi) continue;
        // item complete: write X parts of this wave's index, reset
        const int P = 2 * cPp + pi;
#pragma unroll
        for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int mi = 0; mi < MT; ++mi) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int mu = 128 * cI2 + 32 * rg + 16 * f + 4 * lk + r, i = 16 * mi + li;
                    if (P < n_aux && mu < 64 * nt && i < n_occ) {
                        __bf16 pt[3];
                        split_parts(acc[f][mi][r] + (double)corr[f][mi][r], NS, pt);
                        const int64_t o = (int64_t)mu * R + (int64_t)P * n_occ + i;
#pragma unroll
                        for (int k = 0; k < NS; ++k) Xb[k * xplane + o] = pt[k];
                    }
                }
                acc[f][mi] = d4_t{0, 0, 0, 0};
                corr[f][mi] = f4_t{0.f, 0.f, 0.f, 0.f};
            }
        if (++cj == mine) break;
        cs = 0;
        const int item = (int)blockIdx.x + cj * G;
        cI2 = item % nt2;
        cPp = item / nt2;
    }
    wait_vm<0>();
#endif
}

// K partials over lower 128 x 128 tiles, split over the K index in multiples
// of 32: part[z][mu][nu] = sum_r X[mu][r] X[nu][r] (split products).  Wave w
// owns rows 64 (w % 2) .. +63 and columns 32 (w / 2) .. +31 of the tile.
template <int NS>
__global__ __launch_bounds__(512, 1) void syrk_bf16_kernel(const __bf16* __restrict__ Xb, int Npad, int64_t R,
                                                           int64_t chunk, int ntile, double* __restrict__ part) {
#if defined(__HIP_DEVICE_COMPILE__)   // buffer resources exist on the device side only
    constexpr int SA = NS * 128 * ROWB, STAGE = 2 * SA;
    constexpr int LOADS = 2 * NS * 8 / 8;
    __shared__ __attribute__((aligned(16))) __bf16 ring[RING * STAGE];
    const int nlow = ntile * (ntile + 1) / 2;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int z = L / nlow, t = L % nlow;
    int ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    const int tj = t - ti * (ti + 1) / 2;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lrow = lane >> 2, lch = lane & 3;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 32;
    const int64_t r0 = (int64_t)z * chunk, r1 = min(R, r0 + chunk);
    const int nst = (int)((r1 - r0) / ROWB);
    const int64_t xplane = (int64_t)Npad * R;

    const __bf16* src[LOADS];
    int dst[LOADS];
#pragma unroll
    for (int u = 0; u < LOADS; ++u) {
        const int tt = wave + 8 * u, side = tt / (NS * 8), rem = tt % (NS * 8), p = rem >> 3, rg = rem & 7;
        const int row = 16 * rg + lrow;
        const int base = side ? tj * 128 : ti * 128;
        src[u] = Xb + p * xplane + (int64_t)(base + row) * R + r0 + 8 * swz(row, lch);
        dst[u] = side * SA + (p * 128 + 16 * rg) * ROWB;
    }
    int is = 0;
    auto issue = [&](int slot) {
        __bf16* st = ring + slot * STAGE;
        const int64_t off = (int64_t)is * ROWB;
#pragma unroll
        for (int u = 0; u < LOADS; ++u)
            __builtin_amdgcn_global_load_lds((const void*)(src[u] + off), (lds_void_t)(st + dst[u]), 16, 0, 0);
        if (is + 1 < nst) ++is;                    // tail: reload the last stage (never read)
    };

    d4_t acc[4][2];
    f4_t corr[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { acc[i][j] = d4_t{0, 0, 0, 0}; corr[i][j] = f4_t{0.f, 0.f, 0.f, 0.f}; }
    int s = 0;
    auto body = [&](int slot) -> bool {
        wait_vm<LOADS>();
        __builtin_amdgcn_s_barrier();
        issue(slot == 0 ? 2 : slot - 1);
        const __bf16* sa = ring + slot * STAGE;
        const __bf16* sbb = sa + SA;
        bf8_t a[4][NS], b[2][NS];
#pragma unroll
        for (int p = 0; p < NS; ++p) {
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i][p] = lds_frag(sa + p * 128 * ROWB, wm + 16 * i + li, lk);
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j][p] = lds_frag(sbb + p * 128 * ROWB, wn + 16 * j + li, lk);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) split_mfma<NS>(a[i], b[j], acc[i][j], corr[i][j]);
        if ((s & 7) == 7) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) fold(acc[i][j], corr[i][j]);
        }
        return ++s == nst;
    };
    if (nst > 0) {
        issue(0);
        issue(1);
        while (true) {
            if (body(0)) break;
            if (body(1)) break;
            if (body(2)) break;
        }
        wait_vm<0>();
    }
    double* out = part + (int64_t)z * Npad * Npad;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(int64_t)(ti * 128 + wm + 16 * i + 4 * lk + r) * Npad + tj * 128 + wn + 16 * j + li] =
                    acc[i][j][r] + (double)corr[i][j][r];
#endif
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
    // items of two auxiliary indices each (one C slice per stage serves both)
    const int64_t n_items = (int64_t)((nt + 1) / 2) * ((n_aux + 1) / 2);
    const unsigned grid = (unsigned)std::min<int64_t>(n_items, device_cus());
    const __bf16* b = (const __bf16*)B;
#define XB(NS, M) case M: x_bf16p_kernel<NS, M><<<grid, 512, 0, st>>>(b, nt, n_aux, ct, Npad, n_occ, xb, R); break;
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
    if (ns == 3) syrk_bf16_kernel<3><<<nlow * used, 512, 0, st>>>(xb, Npad, R, chunk, t128, part);
    else syrk_bf16_kernel<2><<<nlow * used, 512, 0, st>>>(xb, Npad, R, chunk, t128, part);
    RI_TRY(hipGetLastError());
    dim3 g2((N + 255) / 256, N);
    kreduce_bf_kernel<<<g2, 256, 0, st>>>(part, used, Npad, N, K);
    return hipGetLastError();
}

}  // namespace ri
