// Integral kernels over normalised primitive s-Gaussians: Schwarz pair
// screening with ordered compaction, three-centre ERIs over significant
// pairs, the two-centre metric, one-electron S and h, nuclear repulsion.
#include "common.h"
#include "kernels.h"

namespace {

constexpr double TWO_PI_52 = 34.98683665524972;   // 2 pi^{5/2}

struct PairC {
    double p, Px, Py, Pz, kn;   // exponent sum, product centre, N_a N_b K_ab
};

__device__ __forceinline__ PairC pair_consts(const double* xyz, const int32_t* fc, const double* fe,
                                             int mu, int nu) {
    double a = fe[mu], b = fe[nu];
    const double* A = xyz + 3 * fc[mu];
    const double* B = xyz + 3 * fc[nu];
    double p = a + b, ip = 1.0 / p;
    double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
    double r2 = dx * dx + dy * dy + dz * dz;
    PairC c;
    c.p = p;
    c.Px = (a * A[0] + b * B[0]) * ip;
    c.Py = (a * A[1] + b * B[1]) * ip;
    c.Pz = (a * A[2] + b * B[2]) * ip;
    c.kn = norm_s(a) * norm_s(b) * exp(-a * b * ip * r2);
    return c;
}

// (mu nu|mu nu) for an s pair: (N_a N_b K)^2 2 pi^{5/2} / (p^2 sqrt(2p)).
__device__ __forceinline__ double schwarz_q(const double* xyz, const int32_t* fc, const double* fe,
                                            int mu, int nu) {
    PairC c = pair_consts(xyz, fc, fe, mu, nu);
    return c.kn * c.kn * TWO_PI_52 / (c.p * c.p * sqrt(2.0 * c.p));
}

__global__ __launch_bounds__(256) void screen_count_kernel(const double* xyz, const int32_t* fc,
                                                           const double* fe, int N, double tau,
                                                           int32_t* counts) {
    const int mu = blockIdx.x;
    int c = 0;
    for (int nu = threadIdx.x; nu <= mu; nu += blockDim.x)
        c += schwarz_q(xyz, fc, fe, mu, nu) > tau;
    __shared__ int sh[4];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) counts[mu] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Exclusive scan of the per-row counts (single thread; N is small).
__global__ void scan_kernel(const int32_t* counts, int N, int64_t* offsets) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t s = 0;
    for (int i = 0; i < N; ++i) {
        offsets[i] = s;
        s += counts[i];
    }
    offsets[N] = s;
}

// Ordered compaction of row mu: pairs (mu, nu), nu ascending.
__global__ __launch_bounds__(256) void screen_write_kernel(const double* xyz, const int32_t* fc,
                                                           const double* fe, int N, double tau,
                                                           const int64_t* offsets, int32_t* pairs) {
    const int mu = blockIdx.x;
    __shared__ int wcount[4];
    __shared__ int64_t base;
    if (threadIdx.x == 0) base = offsets[mu];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int c0 = 0; c0 <= mu; c0 += 256) {
        int nu = c0 + threadIdx.x;
        bool keep = (nu <= mu) && schwarz_q(xyz, fc, fe, mu, nu) > tau;
        uint64_t mask = __ballot(keep);
        int before = __popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
        __syncthreads();
        if (lane == 0) wcount[w] = __popcll(mask);
        __syncthreads();
        int wb = 0;
        for (int i = 0; i < w; ++i) wb += wcount[i];
        if (keep) {
            int64_t idx = base + wb + before;
            pairs[2 * idx] = mu;
            pairs[2 * idx + 1] = nu;
        }
        __syncthreads();
        if (threadIdx.x == 0) base += wcount[0] + wcount[1] + wcount[2] + wcount[3];
        __syncthreads();
    }
}

constexpr int PCH = 32;

// T[P][pair] = N_P 2 pi^{5/2} / (p alpha sqrt(p + alpha)) N_a N_b K_ab
//              F0(p alpha / (p + alpha) |P_ab - R_P|^2)
__global__ __launch_bounds__(256) void eri3_kernel(const double* xyz, const int32_t* fc,
                                                   const double* fe, const int32_t* ac,
                                                   const double* ae, int n_aux,
                                                   const int32_t* pairs, int64_t n_pairs,
                                                   double* T) {
    __shared__ double sa[PCH], sn[PCH], sx[PCH], sy[PCH], sz[PCH];
    const int p0 = blockIdx.y * PCH;
    if (threadIdx.x < PCH && p0 + threadIdx.x < n_aux) {
        int P = p0 + threadIdx.x;
        double al = ae[P];
        sa[threadIdx.x] = al;
        sn[threadIdx.x] = norm_s(al);
        const double* R = xyz + 3 * ac[P];
        sx[threadIdx.x] = R[0];
        sy[threadIdx.x] = R[1];
        sz[threadIdx.x] = R[2];
    }
    __syncthreads();
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    PairC c = pair_consts(xyz, fc, fe, pairs[2 * q], pairs[2 * q + 1]);
    const int np = min(PCH, n_aux - p0);
    for (int k = 0; k < np; ++k) {
        double al = sa[k], s = c.p + al;
        double dx = c.Px - sx[k], dy = c.Py - sy[k], dz = c.Pz - sz[k];
        double t = c.p * al / s * (dx * dx + dy * dy + dz * dz);
        T[(int64_t)(p0 + k) * n_pairs + q] = sn[k] * TWO_PI_52 / (c.p * al * sqrt(s)) * c.kn * boys_f0(t);
    }
}

// A[P][Q] = N_P N_Q 2 pi^{5/2} / (alpha beta sqrt(alpha+beta)) F0(...)
__global__ void metric_kernel(const double* xyz, const int32_t* ac, const double* ae, int n_aux,
                              double* A) {
    int Q = blockIdx.x * blockDim.x + threadIdx.x, P = blockIdx.y;
    if (Q >= n_aux) return;
    double a = ae[P], b = ae[Q], s = a + b;
    const double* R = xyz + 3 * ac[P];
    const double* S = xyz + 3 * ac[Q];
    double dx = R[0] - S[0], dy = R[1] - S[1], dz = R[2] - S[2];
    double t = a * b / s * (dx * dx + dy * dy + dz * dz);
    A[(int64_t)P * n_aux + Q] = norm_s(a) * norm_s(b) * TWO_PI_52 / (a * b * sqrt(s)) * boys_f0(t);
}

// S, h = T + V over all (mu, nu).
__global__ void one_electron_kernel(const double* xyz, const double* Z, int nc, const int32_t* fc,
                                    const double* fe, int N, double* S, double* H) {
    int nu = blockIdx.x * blockDim.x + threadIdx.x, mu = blockIdx.y;
    if (nu >= N) return;
    double a = fe[mu], b = fe[nu];
    const double* A = xyz + 3 * fc[mu];
    const double* B = xyz + 3 * fc[nu];
    double p = a + b, ip = 1.0 / p, m = a * b * ip;
    double dx = A[0] - B[0], dy = A[1] - B[1], dz = A[2] - B[2];
    double r2 = dx * dx + dy * dy + dz * dz;
    double kn = norm_s(a) * norm_s(b) * exp(-m * r2);
    double s = kn * pow(RI_PI * ip, 1.5);
    double t = m * (3.0 - 2.0 * m * r2) * s;
    double Px = (a * A[0] + b * B[0]) * ip, Py = (a * A[1] + b * B[1]) * ip, Pz = (a * A[2] + b * B[2]) * ip;
    double v = 0.0;
    for (int c = 0; c < nc; ++c) {
        double zc = Z[c];
        if (zc == 0.0) continue;
        const double* C = xyz + 3 * c;
        double ex = Px - C[0], ey = Py - C[1], ez = Pz - C[2];
        v -= zc * boys_f0(p * (ex * ex + ey * ey + ez * ez));
    }
    v *= 2.0 * RI_PI * ip * kn;
    S[(int64_t)mu * N + nu] = s;
    H[(int64_t)mu * N + nu] = t + v;
}

__global__ __launch_bounds__(256) void enuc_kernel(const double* xyz, const double* Z, int nc,
                                                   double* out) {
    double e = 0.0;
    for (int64_t k = threadIdx.x; k < (int64_t)nc * nc; k += blockDim.x) {
        int A = k / nc, B = k % nc;
        if (B <= A || Z[A] * Z[B] == 0.0) continue;
        double dx = xyz[3 * A] - xyz[3 * B], dy = xyz[3 * A + 1] - xyz[3 * B + 1],
               dz = xyz[3 * A + 2] - xyz[3 * B + 2];
        e += Z[A] * Z[B] / sqrt(dx * dx + dy * dy + dz * dz);
    }
    __shared__ double sh[4];
    for (int o = 32; o > 0; o >>= 1) e += __shfl_down(e, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) *out = sh[0] + sh[1] + sh[2] + sh[3];
}

}  // namespace

namespace ri {

hipError_t screen_pairs(const ri_system* s, double tau, int32_t* counts, int64_t* offsets,
                        hipStream_t st) {
    screen_count_kernel<<<s->n_fn, 256, 0, st>>>(s->xyz, s->fn_centre, s->fn_exp, s->n_fn, tau, counts);
    RI_TRY(hipGetLastError());
    scan_kernel<<<1, 64, 0, st>>>(counts, s->n_fn, offsets);
    return hipGetLastError();
}

hipError_t write_pairs(const ri_system* s, double tau, const int64_t* offsets, int32_t* pairs,
                       hipStream_t st) {
    screen_write_kernel<<<s->n_fn, 256, 0, st>>>(s->xyz, s->fn_centre, s->fn_exp, s->n_fn, tau, offsets, pairs);
    return hipGetLastError();
}

hipError_t eri3(const ri_system* s, const int32_t* pairs, int64_t n_pairs, double* T, hipStream_t st) {
    if (n_pairs == 0) return hipSuccess;
    dim3 grid((unsigned)((n_pairs + 255) / 256), (s->n_aux + PCH - 1) / PCH);
    eri3_kernel<<<grid, 256, 0, st>>>(s->xyz, s->fn_centre, s->fn_exp, s->aux_centre, s->aux_exp,
                                      s->n_aux, pairs, n_pairs, T);
    return hipGetLastError();
}

hipError_t metric(const ri_system* s, double* A, hipStream_t st) {
    dim3 grid((s->n_aux + 255) / 256, s->n_aux);
    metric_kernel<<<grid, 256, 0, st>>>(s->xyz, s->aux_centre, s->aux_exp, s->n_aux, A);
    return hipGetLastError();
}

hipError_t one_electron(const ri_system* s, double* S, double* H, hipStream_t st) {
    dim3 grid((s->n_fn + 255) / 256, s->n_fn);
    one_electron_kernel<<<grid, 256, 0, st>>>(s->xyz, s->Z, s->n_centres, s->fn_centre, s->fn_exp,
                                              s->n_fn, S, H);
    return hipGetLastError();
}

hipError_t nuclear_repulsion(const ri_system* s, double* out, hipStream_t st) {
    enuc_kernel<<<1, 256, 0, st>>>(s->xyz, s->Z, s->n_centres, out);
    return hipGetLastError();
}

}  // namespace ri
