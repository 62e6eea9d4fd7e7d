// RI-HF analytic gradient contractions: one-electron (D h' - W S'),
// two-centre metric (-1/2 Z (P|Q)'), three-centre (Y (mu nu|P)') and the
// nuclear repulsion derivative.  Derivative integrals are evaluated on the
// fly and accumulated per atom: per-block LDS sums, one partial row per
// block, then a deterministic row reduction.
#include "kernels.h"

#include <algorithm>

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

// sum over all (mu, nu) of D h'_mu_nu - W S'_mu_nu.
__global__ __launch_bounds__(256) void g1e_kernel(const double* xyz, const double* Z, int nc, const int32_t* fc,
                                                  const double* fe, int N, const double* D, const double* W,
                                                  double* part) {
    __shared__ double g[3 * MAXC];
    for (int i = threadIdx.x; i < 3 * nc; i += 256) g[i] = 0.0;
    __syncthreads();
    const int64_t total = (int64_t)N * N;
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        int mu = e / N, nu = e % N;
        double d = D[e], w = W[e];
        double a = fe[mu], b = fe[nu];
        int ca = fc[mu], cb = fc[nu];
        const double* A = xyz + 3 * ca;
        const double* B = xyz + 3 * cb;
        double p = a + b, ip = 1.0 / p, m = a * b * ip;
        double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
        double r2 = dx * dx + dy * dy + dz * dz;
        double kn = norm_s(a) * norm_s(b) * exp(-m * r2);
        // every term of this pair carries kn times D or W: below 1e-24 the pair
        // changes no gradient component by more than ~1e-20 (1e-14 over 1e6 pairs)
        if (kn * (fabs(d) + fabs(w)) < 1e-24) continue;
        double s = kn * pow(RI_PI * ip, 1.5);
        double t = m * (3.0 - 2.0 * m * r2) * s;
        // dS/dA = -2 m (A-B) S ; dT/dA = -2 m (A-B) (2 m S + T)
        double fS = -2.0 * m * s, fT = -2.0 * m * (2.0 * m * s + t);
        double coef = d * fT - w * fS;
        double gx = coef * dx, gy = coef * dy, gz = coef * dz;   // to atom of mu; minus to atom of nu
        double Px = (a * A[0] + b * B[0]) * ip, Py = (a * A[1] + b * B[1]) * ip, Pz = (a * A[2] + b * B[2]) * ip;
        double ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
        const double pre0 = 2.0 * RI_PI * ip * kn;
        for (int c = 0; c < nc; ++c) {
            double zc = Z[c];
            if (zc == 0.0) continue;
            const double* Cc = xyz + 3 * c;
            double ex = Px - Cc[0], ey = Py - Cc[1], ez = Pz - Cc[2];
            double x = p * (ex * ex + ey * ey + ez * ez);
            double pre = zc * pre0;
            double V = -pre * boys_f0(x);
            double f1 = pre * boys_f1(x);
            // dV/dA = V (-2 m (A-B)) + f1 2a (P-C);  dV/dB = V (2 m (A-B)) + f1 2b (P-C);  dV/dC = -f1 2p (P-C)
            double va = -2.0 * m * V;
            ax += d * (va * dx + f1 * 2.0 * a * ex);
            ay += d * (va * dy + f1 * 2.0 * a * ey);
            az += d * (va * dz + f1 * 2.0 * a * ez);
            bx += d * (-va * dx + f1 * 2.0 * b * ex);
            by += d * (-va * dy + f1 * 2.0 * b * ey);
            bz += d * (-va * dz + f1 * 2.0 * b * ez);
            double cc = -d * f1 * 2.0 * p;
            lds_add3(g, c, cc * ex, cc * ey, cc * ez);
        }
        lds_add3(g, ca, gx + ax, gy + ay, gz + az);
        lds_add3(g, cb, -gx + bx, -gy + by, -gz + bz);
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
// U^P = C Xi^P.  Work items are (P, pair) with pairs fastest.
// Auxiliary indices P0 .. P0 + np - 1: WY[P - P0][mu][nu] = (U^P C^T)_mu_nu
// (mu >= nu); contributions are added to the block's partial row.
__global__ __launch_bounds__(256) void g3c_kernel(const double* xyz, const int32_t* fc, const double* fe,
                                                  const int32_t* ac, const double* ae, int P0, int np, int nc,
                                                  const int32_t* pairs, int64_t n_pairs, const double* WY,
                                                  const double* D, int N, const double* cv, double* part) {
    __shared__ double g[3 * MAXC];
    for (int i = threadIdx.x; i < 3 * nc; i += 256) g[i] = 0.0;
    __syncthreads();
    const int64_t total = (int64_t)np * n_pairs;
    for (int64_t e = blockIdx.x * 256ll + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int pl = (int)(e / n_pairs), P = P0 + pl;
        int64_t q = e % n_pairs;
        int mu = pairs[2 * q], nu = pairs[2 * q + 1];
        const double v = WY[((int64_t)pl * N + mu) * N + nu];
        double y = (cv[P] * D[(int64_t)mu * N + nu] - 2.0 * v) * (mu == nu ? 1.0 : 2.0);
        double a = fe[mu], b = fe[nu];
        int ca = fc[mu], cb = fc[nu], cp = ac[P];
        const double* A = xyz + 3 * ca;
        const double* B = xyz + 3 * cb;
        const double* R = xyz + 3 * cp;
        double p = a + b, ip = 1.0 / p, m = a * b * ip;
        double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
        double kn = norm_s(a) * norm_s(b) * exp(-m * (dx * dx + dy * dy + dz * dz));
        double al = ae[P], sa = p + al, w = p * al / sa;
        double ex = (a * A[0] + b * B[0]) * ip - R[0], ey = (a * A[1] + b * B[1]) * ip - R[1],
               ez = (a * A[2] + b * B[2]) * ip - R[2];
        double x = w * (ex * ex + ey * ey + ez * ez);
        double c0 = norm_s(al) * TWO_PI_52 / (p * al * sqrt(sa)) * kn;
        double I = c0 * boys_f0(x);
        double gg = c0 * boys_f1(x) * 2.0 * w;
        // dI/dA = -2 m (A-B) I - gg (a/p) (P-R);  dI/dB = 2 m (A-B) I - gg (b/p) (P-R)
        double t1 = -2.0 * m * I * y, ta = -gg * a * ip * y, tb = -gg * b * ip * y;
        double Ax = t1 * dx + ta * ex, Ay = t1 * dy + ta * ey, Az = t1 * dz + ta * ez;
        double Bx = -t1 * dx + tb * ex, By = -t1 * dy + tb * ey, Bz = -t1 * dz + tb * ez;
        lds_add3(g, ca, Ax, Ay, Az);
        lds_add3(g, cb, Bx, By, Bz);
        lds_add3(g, cp, -(Ax + Bx), -(Ay + By), -(Az + Bz));
    }
    flush_add(g, 3 * nc, part);
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

__global__ void greduce_kernel(const double* part, int rows, int nc3, double* grad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc3) return;
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += part[(int64_t)r * nc3 + i];
    grad[i] = s;
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
    g1e_kernel<<<GRAD_BLOCKS, 256, 0, st>>>(s->xyz, s->Z, s->n_centres, s->fn_centre, s->fn_exp, s->n_fn, D, W, part);
    return hipGetLastError();
}
hipError_t grad_metric(const ri_system* s, const double* Zx, const double* c, double* part, hipStream_t st) {
    if (s->n_centres > MAXC) return hipErrorInvalidValue;
    g2c_kernel<<<GRAD_BLOCKS, 256, 0, st>>>(s->xyz, s->aux_centre, s->aux_exp, s->n_aux, s->n_centres, Zx, c, part);
    return hipGetLastError();
}
int grad_slab(int N, int n_aux) {
    const int64_t per = (int64_t)N * N * 8;
    return (int)std::max<int64_t>(1, std::min<int64_t>(n_aux, (int64_t(1) << 30) / per));
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
        RI_TRY(gemm_f64(false, true, N, N, n_occ, 1.0, U + (int64_t)P0 * N * n_occ, n_occ, (int64_t)N * n_occ, C,
                        n_occ, 0, 0.0, WY, N, (int64_t)N * N, np, 0, 1, st));
        g3c_kernel<<<GRAD_BLOCKS, 256, 0, st>>>(s->xyz, s->fn_centre, s->fn_exp, s->aux_centre, s->aux_exp, P0, np,
                                                s->n_centres, pairs, n_pairs, WY, D, N, c, part);
        RI_TRY(hipGetLastError());
    }
    return hipSuccess;
}
hipError_t grad_nuclear(const ri_system* s, double* part, hipStream_t st) {
    gnuc_kernel<<<1, 256, 0, st>>>(s->xyz, s->Z, s->n_centres, part);
    return hipGetLastError();
}
hipError_t grad_reduce(const double* part, int rows, int n_centres, double* grad, hipStream_t st) {
    greduce_kernel<<<(3 * n_centres + 255) / 256, 256, 0, st>>>(part, rows, 3 * n_centres, grad);
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
