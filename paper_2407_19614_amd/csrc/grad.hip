// RI-HF analytic gradient contractions: one-electron (D h' - W S'),
// two-centre metric (-1/2 Z (P|Q)'), three-centre (Y (mu nu|P)') and the
// nuclear repulsion derivative.  Derivative integrals are evaluated on the
// fly and accumulated per atom: per-block LDS sums, one partial row per
// block, then a deterministic row reduction.
#include "kernels.h"

#include <algorithm>
#include <climits>

namespace {

constexpr double TWO_PI_52 = 34.98683665524972;   // 2 pi^{5/2}
constexpr int MAXC = 2048;                          // centres held in LDS

__device__ __forceinline__ void lds_add3(double* g, int atom, double x, double y, double z) {
    atomicAdd(&g[3 * atom + 0], x);
    atomicAdd(&g[3 * atom + 1], y);
    atomicAdd(&g[3 * atom + 2], z);
}

__device__ void flush(double* g, int nc3, double* part) {
    __syncthreads();
    double* row = part + (int64_t)blockIdx.x * nc3;
    for (int i = threadIdx.x; i < nc3; i += blockDim.x) row[i] = g[i];
}

// as flush, adding to the block's row (launches over several slabs)
__device__ void flush_add(double* g, int nc3, double* part) {
    __syncthreads();
    double* row = part + (int64_t)blockIdx.x * nc3;
    for (int i = threadIdx.x; i < nc3; i += blockDim.x) row[i] += g[i];
}

// F0(t) and F1(t) together.  Below t = 1, F1 from its Taylor series
// F1(t) = sum_k (-t)^k / (k! (2k + 3)), 19 terms (the first omitted term is
// below 3e-18), and F0 = 2t F1 + exp(-t) (the downward relation, all terms
// positive); above, F0 = (sqrt(pi)/2) erf(sqrt t) / sqrt t and
// F1 = (F0 - exp(-t)) / (2t).  From t = 40 on, erfc(sqrt t) < 1e-18 and
// exp(-t) < 5e-18 relative to F0, so both drop out: F0 = (sqrt(pi)/2) / sqrt t
// and F1 = F0 / (2t).
struct BoysTaylor {
    double c[19];
    constexpr BoysTaylor() : c() {
        double f = 1.0;   // (-1)^k / k!
        for (int k = 0; k < 19; ++k) {
            c[k] = f / (2 * k + 3);
            f = -f / (k + 1);
        }
    }
};
__device__ __forceinline__ void boys_f01(double t, double& f0, double& f1) {
    if (t < 1.0) {
        constexpr BoysTaylor B{};
        double s = B.c[18];
#pragma unroll
        for (int k = 17; k >= 0; --k) s = fma(s, t, B.c[k]);
        f1 = s;
        f0 = fma(2.0 * t, s, exp(-t));
    } else if (t < 40.0) {
        const double r = sqrt(t);
        f0 = 0.88622692545275801365 * erf(r) / r;
        f1 = (f0 - exp(-t)) / (2.0 * t);
    } else {
        f0 = 0.88622692545275801365 / sqrt(t);
        f1 = f0 / (2.0 * t);
    }
}

// Sum over the wave; every lane receives the total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// sum over all (mu, nu) of D h'_mu_nu - W S'_mu_nu, taken over mu >= nu with
// weight 2 off the diagonal (h, S, D and W are symmetric).  One lower pair
// per thread; the nuclear-attraction loop over centres is uniform across the
// wave, so each centre's share is summed over the wave before one LDS add.
// g holds 3 * nc doubles of dynamic LDS.
__global__ __launch_bounds__(256) void g1e_kernel(const double* xyz, const double* Z, int nc, const int32_t* fc,
                                                  const double* fe, int N, const double* D, const double* W,
                                                  double* part) {
    extern __shared__ double g[];
    for (int i = threadIdx.x; i < 3 * nc; i += 256) g[i] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t total = (int64_t)N * (N + 1) / 2;
    const int64_t span = (int64_t)gridDim.x * 256;
    const int64_t rounds = (total + span - 1) / span;   // every wave runs the same count: shuffles stay uniform
    for (int64_t r = 0; r < rounds; ++r) {
        const int64_t e = r * span + blockIdx.x * 256ll + threadIdx.x;
        const bool in = e < total;
        int mu = 0, nu = 0;
        if (in) {
            mu = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
            while ((int64_t)(mu + 1) * (mu + 2) / 2 <= e) ++mu;
            while ((int64_t)mu * (mu + 1) / 2 > e) --mu;
            nu = (int)(e - (int64_t)mu * (mu + 1) / 2);
        }
        const double wq = in ? (mu == nu ? 1.0 : 2.0) : 0.0;
        const double d = wq * D[(int64_t)mu * N + nu], w = wq * W[(int64_t)mu * N + nu];
        const double a = fe[mu], b = fe[nu];
        const int ca = fc[mu], cb = fc[nu];
        const double* A = xyz + 3 * ca;
        const double* B = xyz + 3 * cb;
        const double p = a + b, ip = 1.0 / p, m = a * b * ip;
        const double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double kn = norm_s(a) * norm_s(b) * exp(-m * r2);
        // every term of this pair carries kn times D or W: below 1e-24 the pair
        // changes no gradient component by more than ~1e-20 (1e-14 over 1e6 pairs)
        const bool live = in && !(kn * (fabs(d) + fabs(w)) < 1e-24 * wq);
        if (__ballot(live) == 0) continue;
        const double s = kn * pow(RI_PI * ip, 1.5);
        const double t = m * (3.0 - 2.0 * m * r2) * s;
        // dS/dA = -2 m (A-B) S ; dT/dA = -2 m (A-B) (2 m S + T)
        const double fS = -2.0 * m * s, fT = -2.0 * m * (2.0 * m * s + t);
        const double coef = live ? d * fT - w * fS : 0.0;
        const double gx = coef * dx, gy = coef * dy, gz = coef * dz;   // to atom of mu; minus to atom of nu
        const double Px = (a * A[0] + b * B[0]) * ip, Py = (a * A[1] + b * B[1]) * ip, Pz = (a * A[2] + b * B[2]) * ip;
        const double dl = live ? d : 0.0;
        double ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
        const double pre0 = 2.0 * RI_PI * ip * kn;
        for (int c = 0; c < nc; ++c) {
            const double zc = Z[c];
            if (zc == 0.0) continue;
            const double* Cc = xyz + 3 * c;
            const double ex = Px - Cc[0], ey = Py - Cc[1], ez = Pz - Cc[2];
            const double x = p * (ex * ex + ey * ey + ez * ez);
            const double pre = zc * pre0;
            double F0, F1;
            boys_f01(x, F0, F1);
            const double V = -pre * F0;
            const double f1 = pre * F1;
            // dV/dA = V (-2 m (A-B)) + f1 2a (P-C);  dV/dB = V (2 m (A-B)) + f1 2b (P-C);  dV/dC = -f1 2p (P-C)
            const double va = -2.0 * m * V;
            ax += dl * (va * dx + f1 * 2.0 * a * ex);
            ay += dl * (va * dy + f1 * 2.0 * a * ey);
            az += dl * (va * dz + f1 * 2.0 * a * ez);
            bx += dl * (-va * dx + f1 * 2.0 * b * ex);
            by += dl * (-va * dy + f1 * 2.0 * b * ey);
            bz += dl * (-va * dz + f1 * 2.0 * b * ez);
            const double cc = -dl * f1 * 2.0 * p;
            const double sx = wave_sum(cc * ex), sy = wave_sum(cc * ey), sz = wave_sum(cc * ez);
            if (lane == 0) lds_add3(g, c, sx, sy, sz);
        }
        if (live) {
            lds_add3(g, ca, gx + ax, gy + ay, gz + az);
            lds_add3(g, cb, -gx + bx, -gy + by, -gz + bz);
        }
    }
    flush(g, 3 * nc, part);
}

// -1/2 sum_PQ Z_PQ (P|Q)' over the lower triangle (P > Q, weight 2);
// Z_PQ = c_P c_Q + Zx_PQ where Zx (lower) holds -2 sum_ij Xi Xi.
__global__ __launch_bounds__(256) void g2c_kernel(const double* xyz, const int32_t* ac, const double* ae, int na,
                                                  int nc, const double* Zx, const double* cv, double* part) {
    __shared__ double g[3 * MAXC];
    for (int i = threadIdx.x; i < 3 * nc; i += 256) g[i] = 0.0;
    __syncthreads();
    const int64_t total = (int64_t)na * na;
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int P = e / na, Q = e % na;
        if (Q >= P) continue;
        int cp = ac[P], cq = ac[Q];
        if (cp == cq) continue;
        double z = Zx[e] + cv[P] * cv[Q];
        double a = ae[P], b = ae[Q], s = a + b, w = a * b / s;
        const double* R = xyz + 3 * cp;
        const double* S = xyz + 3 * cq;
        double dx = R[0] - S[0], dy = R[1] - S[1], dz = R[2] - S[2];
        double c0 = norm_s(a) * norm_s(b) * TWO_PI_52 / (a * b * sqrt(s));
        double f = -c0 * boys_f1(w * (dx * dx + dy * dy + dz * dz)) * 2.0 * w;   // d(P|Q)/dR_P / (R_P - R_Q)
        double k = -z * f;   // -1/2 * 2 * Z * f
        lds_add3(g, cp, k * dx, k * dy, k * dz);
        lds_add3(g, cq, -k * dx, -k * dy, -k * dz);
    }
    flush(g, 3 * nc, part);
}

// sum_P sum_pairs w Y^P_mu_nu (mu nu|P)',  Y = c_P D_mu_nu - 2 (U^P C^T)_mu_nu,
// U^P = C Xi^P.  Auxiliary indices P0 .. P0 + np - 1: WY[P - P0][mu][nu] =
// (U^P C^T)_mu_nu (mu >= nu); contributions are added to the block's partial
// row.  Work items are (block of 256 pairs, chunk of G3_PC auxiliaries): one
// pair per thread, its Gaussian product and prefactor formed once, then the
// chunk's auxiliaries in turn (their exponents, normalisation and centres
// staged in LDS).  The pair's two centres accumulate in registers; the
// auxiliary's centre is the same for the whole wave at each step, so its
// share is summed over the wave before one LDS add.  g holds 3 * nc doubles
// of dynamic LDS.
constexpr int G3_PC = 8;

__global__ __launch_bounds__(256) void g3c_kernel(const double* xyz, const int32_t* fc, const double* fe,
                                                  const int32_t* ac, const double* ae, int P0, int np, int nc,
                                                  const int32_t* pairs, int64_t n_pairs, const double* WY,
                                                  const double* D, int N, const double* cv, double* part) {
    extern __shared__ double g[];
    __shared__ double sp[G3_PC][6];   // alpha, norm(alpha) / alpha, centre (3), c_P
    __shared__ int sc[G3_PC];
    const int tid = threadIdx.x, lane = tid & 63;
    for (int i = tid; i < 3 * nc; i += 256) g[i] = 0.0;
    const int64_t pb = (n_pairs + 255) / 256;
    const int64_t items = pb * ((np + G3_PC - 1) / G3_PC);
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int pc0 = (int)(it / pb) * G3_PC, pcn = min(G3_PC, np - pc0);
        const int64_t q = (it % pb) * 256 + tid;
        __syncthreads();   // the previous item's reads of sp are done (g zeroed before the first)
        if (tid < pcn) {
            const int P = P0 + pc0 + tid, c = ac[P];
            const double al = ae[P];
            sp[tid][0] = al;
            sp[tid][1] = norm_s(al) / al;
            sp[tid][2] = xyz[3 * c];
            sp[tid][3] = xyz[3 * c + 1];
            sp[tid][4] = xyz[3 * c + 2];
            sp[tid][5] = cv[P];
            sc[tid] = c;
        }
        __syncthreads();
        const bool live = q < n_pairs;
        int mu = 0, nu = 0;
        if (live) {
            mu = pairs[2 * q];
            nu = pairs[2 * q + 1];
        }
        const double wq = live ? (mu == nu ? 1.0 : 2.0) : 0.0;   // lanes past the pairs add zeros
        const double dmn = D[(int64_t)mu * N + nu];
        const double a = fe[mu], b = fe[nu];
        const int ca = fc[mu], cb = fc[nu];
        const double* A = xyz + 3 * ca;
        const double* B = xyz + 3 * cb;
        const double p = a + b, ip = 1.0 / p, m = a * b * ip;
        const double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
        // c0 = norm(a) norm(b) norm(alpha) exp(-m |A-B|^2) 2 pi^{5/2} / (p alpha sqrt(p + alpha))
        const double kp = norm_s(a) * norm_s(b) * exp(-m * (dx * dx + dy * dy + dz * dz)) * TWO_PI_52 * ip;
        const double Px = (a * A[0] + b * B[0]) * ip, Py = (a * A[1] + b * B[1]) * ip, Pz = (a * A[2] + b * B[2]) * ip;
        const double* wy = WY + ((int64_t)pc0 * N + mu) * N + nu;
        double gax = 0, gay = 0, gaz = 0, gbx = 0, gby = 0, gbz = 0;
        for (int k = 0; k < pcn; ++k) {
            const double al = sp[k][0];
            const double y = (sp[k][5] * dmn - 2.0 * wy[(int64_t)k * N * N]) * wq;
            const double isa = 1.0 / (p + al), w = p * al * isa;
            const double ex = Px - sp[k][2], ey = Py - sp[k][3], ez = Pz - sp[k][4];
            double F0, F1;
            boys_f01(w * (ex * ex + ey * ey + ez * ez), F0, F1);
            const double c0 = kp * sp[k][1] * sqrt(isa);
            const double I = c0 * F0, gg = c0 * F1 * 2.0 * w;
            // dI/dA = -2 m (A-B) I - gg (a/p) (P-R);  dI/dB = 2 m (A-B) I - gg (b/p) (P-R)
            const double t1 = -2.0 * m * I * y, ta = -gg * a * ip * y, tb = -gg * b * ip * y;
            const double Ax = t1 * dx + ta * ex, Ay = t1 * dy + ta * ey, Az = t1 * dz + ta * ez;
            const double Bx = -t1 * dx + tb * ex, By = -t1 * dy + tb * ey, Bz = -t1 * dz + tb * ez;
            gax += Ax; gay += Ay; gaz += Az;
            gbx += Bx; gby += By; gbz += Bz;
            const double sx = wave_sum(Ax + Bx), sy = wave_sum(Ay + By), sz = wave_sum(Az + Bz);
            if (lane == 0) lds_add3(g, sc[k], -sx, -sy, -sz);
        }
        if (live) {
            lds_add3(g, ca, gax, gay, gaz);
            lds_add3(g, cb, gbx, gby, gbz);
        }
    }
    flush_add(g, 3 * nc, part);
}

// WY[p][mu][nu] = sum_i U[p][mu][i] C[nu][i] on the lower 64 x 64 tiles
// (mu, nu < N) for p in [0, np); U [np][N][K], C [N][K] row-major, K <= 8 KU.
// One workgroup per (lower tile (I, J), group of WY_PB auxiliaries); each of
// the 4 waves owns 32 x 32 of the tile as 2 x 2 FP64 MFMA blocks.  The tile
// column's 64 rows of C stay in registers as B operands for the whole group;
// U's rows stream from memory 16 B per lane.  MFMA step 2u + h of a lane in
// group g (lanes 16 g ..) takes reduction index 8u + 2g + h, the same order
// on both operands; indices >= K are zeroed in registers (a row's tail would
// read the next row), and rows >= N read as zero through the buffer range.
constexpr int WY_PB = 8;

template <int KU>
__global__ __launch_bounds__(256, 2) void wy_kernel(const double* __restrict__ U, const double* __restrict__ C,
                                                    int N, int K, int np, double* __restrict__ WY) {
    const int t = blockIdx.x;
    int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int J = t - I * (I + 1) / 2;
    const int p0 = blockIdx.y * WY_PB, p1 = min(np, p0 + WY_PB);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, g = lane >> 4;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int rowbytes = K * 8;
    const __amdgpu_buffer_rsrc_t cr =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(C), (short)0, N * rowbytes, 0x00020000);
    d2_t b[2][KU];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int nu = 64 * J + wn + 16 * j + li;
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int k0 = 8 * u + 2 * g;
            d2_t v = __builtin_bit_cast(d2_t, __builtin_amdgcn_raw_buffer_load_b128(cr, nu * rowbytes + k0 * 8, 0, 0));
            if (k0 >= K) v[0] = 0.0;
            if (k0 + 1 >= K) v[1] = 0.0;
            b[j][u] = v;
        }
    }
    for (int p = p0; p < p1; ++p) {
        const __amdgpu_buffer_rsrc_t ur = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<double*>(U + (int64_t)p * N * K), (short)0, N * rowbytes, 0x00020000);
        d4_t acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
        const int r0 = (64 * I + wm + li) * rowbytes, r1 = r0 + 16 * rowbytes;
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int k0 = 8 * u + 2 * g;
            d2_t a0 = __builtin_bit_cast(d2_t, __builtin_amdgcn_raw_buffer_load_b128(ur, r0 + k0 * 8, 0, 0));
            d2_t a1 = __builtin_bit_cast(d2_t, __builtin_amdgcn_raw_buffer_load_b128(ur, r1 + k0 * 8, 0, 0));
            if (k0 >= K) { a0[0] = 0.0; a1[0] = 0.0; }
            if (k0 + 1 >= K) { a0[1] = 0.0; a1[1] = 0.0; }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[0][j] = mfma_f64(a0[h], b[j][u][h], acc[0][j]);
                    acc[1][j] = mfma_f64(a1[h], b[j][u][h], acc[1][j]);
                }
            }
        }
        double* out = WY + (int64_t)p * N * N;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = 64 * J + wn + 16 * j + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 64 * I + wm + 16 * i + 4 * r + g;
                    if (row < N && col < N) out[(int64_t)row * N + col] = acc[i][j][r];
                }
            }
    }
}

// U[p][mu][i] = sum_j C[mu][j] Xi^p[i][j] for p in [0, np): C [N][K], Xi^p the
// K x K block p of Xi [np][K][K].  Xi^p is symmetric (Xi = L^{-T} B_ij, and
// each B_ij^P = C^T B^P C is), so this is C Xi^p read along its rows.  The
// structure of wy_kernel with the roles swapped: C's 64 rows of the row tile
// stay in registers as A operands for a group of WY_PB auxiliaries, and
// Xi^p's rows stream in as B operands.  Grid: (row tile, column tile of the
// n_occ columns) x groups of auxiliaries.
template <int KU>
__global__ __launch_bounds__(256, 2) void u_kernel(const double* __restrict__ C, const double* __restrict__ Xi,
                                                   int N, int K, int np, double* __restrict__ U) {
    const int nct = (K + 63) / 64;
    const int I = blockIdx.x / nct, Jc = blockIdx.x % nct;
    const int p0 = blockIdx.y * WY_PB, p1 = min(np, p0 + WY_PB);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, g = lane >> 4;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int rowbytes = K * 8;
    const __amdgpu_buffer_rsrc_t cr =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(C), (short)0, N * rowbytes, 0x00020000);
    d2_t a[2][KU];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int mu = 64 * I + wm + 16 * i + li;
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int k0 = 8 * u + 2 * g;
            d2_t v = __builtin_bit_cast(d2_t, __builtin_amdgcn_raw_buffer_load_b128(cr, mu * rowbytes + k0 * 8, 0, 0));
            if (k0 >= K) v[0] = 0.0;
            if (k0 + 1 >= K) v[1] = 0.0;
            a[i][u] = v;
        }
    }
    for (int p = p0; p < p1; ++p) {
        const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<double*>(Xi + (int64_t)p * K * K), (short)0, K * rowbytes, 0x00020000);
        d4_t acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};
        const int r0 = (64 * Jc + wn + li) * rowbytes, r1 = r0 + 16 * rowbytes;
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int k0 = 8 * u + 2 * g;
            d2_t b0 = __builtin_bit_cast(d2_t, __builtin_amdgcn_raw_buffer_load_b128(xr, r0 + k0 * 8, 0, 0));
            d2_t b1 = __builtin_bit_cast(d2_t, __builtin_amdgcn_raw_buffer_load_b128(xr, r1 + k0 * 8, 0, 0));
            if (k0 >= K) { b0[0] = 0.0; b1[0] = 0.0; }
            if (k0 + 1 >= K) { b0[1] = 0.0; b1[1] = 0.0; }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    acc[i][0] = mfma_f64(a[i][u][h], b0[h], acc[i][0]);
                    acc[i][1] = mfma_f64(a[i][u][h], b1[h], acc[i][1]);
                }
            }
        }
        double* out = U + (int64_t)p * N * K;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = 64 * Jc + wn + 16 * j + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 64 * I + wm + 16 * i + 4 * r + g;
                    if (row < N && col < K) out[(int64_t)row * K + col] = acc[i][j][r];
                }
            }
    }
}

__global__ __launch_bounds__(256) void gnuc_kernel(const double* xyz, const double* Z, int nc, double* part) {
    for (int A = threadIdx.x; A < nc; A += 256) {
        double gx = 0, gy = 0, gz = 0;
        for (int B = 0; B < nc; ++B) {
            if (B == A || Z[A] * Z[B] == 0.0) continue;
            double dx = xyz[3 * A] - xyz[3 * B], dy = xyz[3 * A + 1] - xyz[3 * B + 1], dz = xyz[3 * A + 2] - xyz[3 * B + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double f = -Z[A] * Z[B] / (r * r * r);
            gx += f * dx; gy += f * dy; gz += f * dz;
        }
        part[3 * A] = gx; part[3 * A + 1] = gy; part[3 * A + 2] = gz;
    }
}

// grad[i] = sum over rows of part[row][i]: one block per component, the rows
// strided over the threads, then a fixed-order tree (deterministic).
__global__ __launch_bounds__(256) void greduce_kernel(const double* part, int rows, int nc3, double* grad) {
    const int i = blockIdx.x;
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += 256) s += part[(int64_t)r * nc3 + i];
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[i] = sh[0];
}

// out[r][c] = sum_z part[z][r][c] for c <= r, z in order.
__global__ void sum_lower_kernel(const double* part, int S, int64_t stride, int n, double* out) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    if (e % n > e / n) return;
    double s = part[e];
    for (int z = 1; z < S; ++z) s += part[z * stride + e];
    out[e] = s;
}

__global__ void gamma_dp_kernel(const int32_t* pairs, int64_t n_pairs, const double* C, int n_occ, double* dp) {
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    int mu = pairs[2 * q], nu = pairs[2 * q + 1];
    double s = 0.0;
    for (int i = 0; i < n_occ; ++i) s += C[(int64_t)mu * n_occ + i] * C[(int64_t)nu * n_occ + i];
    dp[q] = (mu == nu ? 2.0 : 4.0) * s;
}

__global__ __launch_bounds__(256) void gamma_row_kernel(const double* Bc, int64_t n_pairs, const double* dp,
                                                        double* gamma) {
    const double* row = Bc + (int64_t)blockIdx.x * n_pairs;
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < n_pairs; q += 256) s += row[q] * dp[q];
    __shared__ double sh[4];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) gamma[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

}  // namespace

namespace ri {

hipError_t grad_one_electron(const ri_system* s, const double* D, const double* W, double* part, hipStream_t st) {
    if (s->n_centres > MAXC) return hipErrorInvalidValue;
    g1e_kernel<<<GRAD_BLOCKS, 256, 3 * s->n_centres * sizeof(double), st>>>(s->xyz, s->Z, s->n_centres, s->fn_centre, s->fn_exp, s->n_fn, D, W, part);
    return hipGetLastError();
}
hipError_t grad_metric(const ri_system* s, const double* Zx, const double* c, double* part, hipStream_t st) {
    if (s->n_centres > MAXC) return hipErrorInvalidValue;
    g2c_kernel<<<GRAD_BLOCKS, 256, 0, st>>>(s->xyz, s->aux_centre, s->aux_exp, s->n_aux, s->n_centres, Zx, c, part);
    return hipGetLastError();
}
// Zx = -2 Xi Xi^T on the lower tiles (Xi: n_aux x K, row-major).  The
// reduction over K is split into S column ranges, one batch of the GEMM each,
// into S partial products in `tmp` (tmp_elems doubles), then summed in order:
// the unsplit form has only the lower 128-tiles as workgroups (300 at
// n_aux = 3000), too few to fill the chip for a long K.
hipError_t grad_metric_z(const double* Xi, int n_aux, int64_t K, double* tmp, int64_t tmp_elems, double* Zx,
                         hipStream_t st) {
    const int64_t n2 = (int64_t)n_aux * n_aux;
    const int64_t t128 = (n_aux + 127) / 128, lower = t128 * (t128 + 1) / 2;
    int S = (int)std::max<int64_t>(1, std::min<int64_t>({(3 * 512 + lower / 2) / lower, 16, K / 256, tmp_elems / n2 - 1}));
    if (S <= 1)
        return gemm_f64(false, true, n_aux, n_aux, (int)K, -2.0, Xi, K, 0, Xi, K, 0, 0.0, Zx, n_aux, 0, 1, 0, 1, st);
    // S equal ranges in one launch; the K % S columns left over, if any, in a
    // launch of their own into one more partial
    const int64_t kc = K / S, rem = K - S * kc;
    RI_TRY(gemm_f64(false, true, n_aux, n_aux, (int)kc, -2.0, Xi, K, kc, Xi, K, kc, 0.0, tmp, n_aux, n2, S, 0, 1, st));
    if (rem > 0) {
        RI_TRY(gemm_f64(false, true, n_aux, n_aux, (int)rem, -2.0, Xi + S * kc, K, 0, Xi + S * kc, K, 0, 0.0,
                        tmp + (int64_t)S * n2, n_aux, 0, 1, 0, 1, st));
        ++S;
    }
    sum_lower_kernel<<<(unsigned)((n2 + 255) / 256), 256, 0, st>>>(tmp, S, n2, n_aux, Zx);
    return hipGetLastError();
}
int grad_slab(int N, int n_aux) {
    const int64_t per = (int64_t)N * N * 8;
    return (int)std::max<int64_t>(1, std::min<int64_t>(n_aux, (int64_t(1) << 30) / per));
}

// WY[p] = U^p C^T on the lower 64 x 64 tiles for p < np (U [np][N][K]).
hipError_t wy_products(const double* U, const double* C, int N, int K, int np, double* WY, hipStream_t st) {
    const int ku = (K + 7) / 8, nt = (N + 63) / 64;
    if (ku > 16 || (int64_t)N * K * 8 > INT_MAX)
        return gemm_f64(false, true, N, N, K, 1.0, U, K, (int64_t)N * K, C, K, 0, 0.0, WY, N, (int64_t)N * N, np, 0, 1,
                        st);
    const dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)((np + WY_PB - 1) / WY_PB));
    switch (ku) {
#define WYK(n) case n: wy_kernel<n><<<grid, 256, 0, st>>>(U, C, N, K, np, WY); break;
        WYK(1) WYK(2) WYK(3) WYK(4) WYK(5) WYK(6) WYK(7) WYK(8)
        WYK(9) WYK(10) WYK(11) WYK(12) WYK(13) WYK(14) WYK(15) WYK(16)
#undef WYK
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
// U[p] = C Xi^p for p < np (Xi [np][K][K], each block symmetric; U [np][N][K]).
hipError_t u_products(const double* C, const double* Xi, int N, int K, int np, double* U, hipStream_t st) {
    const int ku = (K + 7) / 8;
    if (ku > 16 || (int64_t)N * K * 8 > INT_MAX)
        return gemm_f64(false, false, N, K, K, 1.0, C, K, 0, Xi, K, (int64_t)K * K, 0.0, U, K, (int64_t)N * K, np, 0,
                        0, st);
    const dim3 grid((unsigned)(((N + 63) / 64) * ((K + 63) / 64)), (unsigned)((np + WY_PB - 1) / WY_PB));
    switch (ku) {
#define UK(n) case n: u_kernel<n><<<grid, 256, 0, st>>>(C, Xi, N, K, np, U); break;
        UK(1) UK(2) UK(3) UK(4) UK(5) UK(6) UK(7) UK(8)
        UK(9) UK(10) UK(11) UK(12) UK(13) UK(14) UK(15) UK(16)
#undef UK
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
hipError_t grad_three_centre(const ri_system* s, const int32_t* pairs, int64_t n_pairs, const double* U,
                             const double* C, int n_occ, const double* D, const double* c, double* WY,
                             double* part, hipStream_t st) {
    if (s->n_centres > MAXC) return hipErrorInvalidValue;
    const int N = s->n_fn, na = s->n_aux, ns = grad_slab(N, na);
    RI_TRY(fill(part, 0.0, (int64_t)GRAD_BLOCKS * 3 * s->n_centres, st));
    if (n_pairs == 0) return hipSuccess;
    for (int P0 = 0; P0 < na; P0 += ns) {
        const int np = std::min(ns, na - P0);
        // WY[p] = U^{P0+p} C^T on the tiles holding mu >= nu
        RI_TRY(wy_products(U + (int64_t)P0 * N * n_occ, C, N, n_occ, np, WY, st));
        g3c_kernel<<<GRAD_BLOCKS, 256, 3 * s->n_centres * sizeof(double), st>>>(
            s->xyz, s->fn_centre, s->fn_exp, s->aux_centre, s->aux_exp, P0, np, s->n_centres, pairs, n_pairs, WY, D,
            N, c, part);
        RI_TRY(hipGetLastError());
    }
    return hipSuccess;
}
hipError_t grad_nuclear(const ri_system* s, double* part, hipStream_t st) {
    gnuc_kernel<<<1, 256, 0, st>>>(s->xyz, s->Z, s->n_centres, part);
    return hipGetLastError();
}
hipError_t grad_reduce(const double* part, int rows, int n_centres, double* grad, hipStream_t st) {
    greduce_kernel<<<3 * n_centres, 256, 0, st>>>(part, rows, 3 * n_centres, grad);
    return hipGetLastError();
}
hipError_t gamma_only(const double* Bc, const int32_t* pairs, int64_t n_pairs, int n_aux, int n_occ, const double* C,
                      double* dpair, double* gamma, hipStream_t st) {
    if (n_pairs == 0) return fill(gamma, 0.0, n_aux, st);
    gamma_dp_kernel<<<(unsigned)((n_pairs + 255) / 256), 256, 0, st>>>(pairs, n_pairs, C, n_occ, dpair);
    RI_TRY(hipGetLastError());
    gamma_row_kernel<<<n_aux, 256, 0, st>>>(Bc, n_pairs, dpair, gamma);
    return hipGetLastError();
}

}  // namespace ri
