// Batched SCF (project extension): many independent molecules advance in
// lockstep.  Every step of an SCF iteration (Fock build, Fock assembly,
// energy, DIIS, purification, occupied space) is one launch over the work
// items of all active molecules (MolDesc + prefix tables, grouped GEMMs), so
// the iteration is a fixed launch sequence that can be captured once as a
// HIP graph and replayed; convergence and DIIS bookkeeping stay on the
// device and the host reads one counter per iteration.
#include "kernels.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace {

using ri::MolDesc;

constexpr int ST_ACTIVE = 0, ST_IT = 1, ST_PUSH = 2, ST_CONV = 3, ST_NSLOT = 4, ST_SLOT0 = 5, ST_BAD = 13;
// purification: ST_TC2 1 while squares are still formed, ST_TC2U 1 if this
// step's update runs, ST_TC2X the steps left once idempotent (-1 before)
constexpr int ST_TC2 = 14, ST_TC2X = 15, ST_TC2U = 16, ST_N = 32;
// ST_NOPUR 1 once a purification ended its launch sequence without reaching the
// idempotency threshold: the molecule stops iterating and is reported unconverged
constexpr int ST_NOPUR = 17;
constexpr int SC_E = 0, SC_ERR = 5, SC_EOLD = 6, SC_ENUC = 8, SC_BOUNDS = 16, SC_TR = 20;

#define DECODE()                                         \
    int mol, loc;                                        \
    ri::decode_item(prefix, n_mol, blockIdx.x, mol, loc); \
    const MolDesc& m = d[mol];                           \
    if (!m.state[ST_ACTIVE]) return;

__device__ __forceinline__ double block_sum256(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return r;
}
__device__ __forceinline__ double block_max256(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

// -------------------------------------------------- elementwise over N x N
// prefix over ceil(N^2 / 256) blocks per molecule
__global__ void fock_assemble_b(const MolDesc* d, const int* prefix, int n_mol) {
    DECODE();
    int64_t e = (int64_t)loc * 256 + threadIdx.x;
    if (e < (int64_t)m.N * m.N) m.F[e] = m.H[e] + m.J[e] - m.K[e];
}

__global__ void copy_h_b(const MolDesc* d, const int* prefix, int n_mol) {
    DECODE();
    int64_t e = (int64_t)loc * 256 + threadIdx.x;
    if (e < (int64_t)m.N * m.N) m.Fx[e] = m.H[e];
}

__global__ void commutator_b(const MolDesc* d, const int* prefix, int n_mol) {
    DECODE();
    int64_t e = (int64_t)loc * 256 + threadIdx.x;
    if (e >= (int64_t)m.N * m.N) return;
    int r = e / m.N, c = e % m.N;
    m.E[e] = m.T2[e] - m.T2[(int64_t)c * m.N + r];
}

// DIIS ring: slot = pushes mod diis_n (the bookkeeping kernel advances it)
__global__ void diis_push_b(const MolDesc* d, const int* prefix, int n_mol) {
    DECODE();
    int64_t e = (int64_t)loc * 256 + threadIdx.x;
    if (e >= (int64_t)m.N * m.N) return;
    const int s = m.state[ST_PUSH] % m.diis_n;
    m.dF[s][e] = m.F[e];
    m.dE[s][e] = m.E[e];
}

__global__ void diis_combine_b(const MolDesc* d, const int* prefix, int n_mol) {
    DECODE();
    int64_t e = (int64_t)loc * 256 + threadIdx.x;
    if (e >= (int64_t)m.N * m.N) return;
    const int ns = m.state[ST_NSLOT];
    double s = 0.0;
    for (int k = 0; k < ns; ++k) s += m.coef[k] * m.dF[m.state[ST_SLOT0 + k]][e];
    m.Fx[e] = s;
}

__global__ void tc2_init_b(const MolDesc* d, const int* prefix, int n_mol) {
    DECODE();
    int64_t e = (int64_t)loc * 256 + threadIdx.x;
    if (e >= (int64_t)m.N * m.N) return;
    int r = e / m.N, c = e % m.N;
    const double lo = m.scal[SC_BOUNDS], hi = m.scal[SC_BOUNDS + 1];
    // symmetrised, so that X and every square of it (formed on the upper tiles
    // and mirrored) stay exactly symmetric
    const double fs = 0.5 * (m.T2[e] + m.T2[(int64_t)c * m.N + r]);
    m.X[e] = ((r == c ? hi : 0.0) - fs) / (hi - lo);
}

// Grid-stride over the molecule's N^2 elements with the blocks its prefix
// table gives it (about N^2 / 2048), so that a step whose molecules have all
// finished costs few empty blocks.
__global__ void tc2_update_b(const MolDesc* d, const int* prefix, int n_mol) {
    DECODE();
    if (!m.state[ST_TC2U]) return;
    const int nblk = prefix[mol + 1] - prefix[mol];
    const double t1 = m.scal[SC_TR], t2 = m.scal[SC_TR + 1];
    const bool sq = fabs(t2 - m.n_occ) < fabs(2.0 * t1 - t2 - m.n_occ);
    const int64_t n = (int64_t)m.N * m.N;
    for (int64_t e = (int64_t)loc * 256 + threadIdx.x; e < n; e += (int64_t)nblk * 256)
        m.X[e] = sq ? m.X2[e] : 2.0 * m.X[e] - m.X2[e];
}

// -------------------------------------------------- one block per molecule
__global__ __launch_bounds__(256) void state_init_b(const MolDesc* d, int n_mol) {
    const MolDesc& m = d[blockIdx.x];
    if (threadIdx.x < ST_N)
        m.state[threadIdx.x] = (threadIdx.x == ST_ACTIVE || threadIdx.x == ST_TC2 || threadIdx.x == ST_TC2U) ? 1
                               : threadIdx.x == ST_TC2X                                                     ? -1
                                                                                                            : 0;
    if (threadIdx.x < 64) m.Bmat[threadIdx.x] = 0.0;
    if (threadIdx.x == 0) m.scal[SC_EOLD] = 0.0;
}

__global__ __launch_bounds__(256) void hash_cp_b(const MolDesc* d, int n_mol) {
    const MolDesc& m = d[blockIdx.x];
    const int64_t n = (int64_t)m.N * m.n_occ;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        uint32_t x = (uint32_t)i * 2654435761u ^ 0x5eed1234u;
        x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
        m.Cp[i] = (double)x * (2.0 / 4294967296.0) - 1.0;
    }
}

// energies E_1e = tr DH, E_J = tr DJ / 2, E_K = -tr DK / 2, then max|e| and
// the convergence decision (|E - E_old| < tol_E and max|e| < tol_err from the
// second iteration on); a molecule that converges or reaches max_iter
// becomes inactive for the rest of the batch.
__global__ __launch_bounds__(256) void energy_conv_b(const MolDesc* d, int n_mol, int max_iter) {
    const MolDesc& m = d[blockIdx.x];
    if (!m.state[ST_ACTIVE]) return;
    __shared__ double sh[4];
    const int64_t n = (int64_t)m.N * m.N;
    double a = 0.0, b = 0.0, c = 0.0, e = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        double dd = m.D[i];
        a += dd * m.H[i];
        b += dd * m.J[i];
        c += dd * m.K[i];
        e = fmax(e, fabs(m.E[i]));
    }
    a = block_sum256(a, sh);
    b = block_sum256(b, sh);
    c = block_sum256(c, sh);
    e = block_max256(e, sh);
    if (threadIdx.x == 0) {
        const double en = m.scal[SC_ENUC];
        const double E = a + 0.5 * b - 0.5 * c + en;
        m.scal[SC_E + 0] = E;
        m.scal[SC_E + 1] = en;
        m.scal[SC_E + 2] = a;
        m.scal[SC_E + 3] = 0.5 * b;
        m.scal[SC_E + 4] = -0.5 * c;
        m.scal[SC_ERR] = e;
        const int it = ++m.state[ST_IT];
        const double dE = E - m.scal[SC_EOLD];
        m.scal[SC_EOLD + 1] = dE;
        if (it > 1 && fabs(dE) < m.tol_E && e < m.tol_err) {
            m.state[ST_CONV] = 1;
            m.state[ST_ACTIVE] = 0;
            m.state[ST_TC2] = 0;
        } else if (it >= max_iter) {
            m.state[ST_ACTIVE] = 0;
            m.state[ST_TC2] = 0;
        }
        m.scal[SC_EOLD] = E;
    }
}

// Final FP64 exchange after an FP32 SCF: every converged molecule takes part
// once more, then the energy is formed from the same D, h and J with the
// rebuilt K and the molecule is left inactive.  A molecule that did not
// converge keeps its FP32 energies.
__global__ void final_begin_b(const MolDesc* d, int n_mol) {
    if (threadIdx.x == 0) d[blockIdx.x].state[ST_ACTIVE] = d[blockIdx.x].state[ST_CONV];
}

__global__ __launch_bounds__(256) void energy_final_b(const MolDesc* d, int n_mol) {
    const MolDesc& m = d[blockIdx.x];
    if (!m.state[ST_ACTIVE]) return;
    __shared__ double sh[4];
    const int64_t n = (int64_t)m.N * m.N;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double dd = m.D[i];
        a += dd * m.H[i];
        b += dd * m.J[i];
        c += dd * m.K[i];
    }
    a = block_sum256(a, sh);
    b = block_sum256(b, sh);
    c = block_sum256(c, sh);
    if (threadIdx.x == 0) {
        const double en = m.scal[SC_ENUC];
        m.scal[SC_E + 0] = a + 0.5 * b - 0.5 * c + en;
        m.scal[SC_E + 1] = en;
        m.scal[SC_E + 2] = a;
        m.scal[SC_E + 3] = 0.5 * b;
        m.scal[SC_E + 4] = -0.5 * c;
        m.state[ST_ACTIVE] = 0;
    }
}

// after the push: advance the ring and keep the slot order (oldest first)
__global__ void diis_book_b(const MolDesc* d, int n_mol) {
    const MolDesc& m = d[blockIdx.x];
    if (threadIdx.x != 0 || !m.state[ST_ACTIVE]) return;
    const int s = m.state[ST_PUSH] % m.diis_n;
    m.state[ST_PUSH] += 1;
    int ns = m.state[ST_NSLOT], w = 0;
    for (int k = 0; k < ns; ++k)
        if (m.state[ST_SLOT0 + k] != s) m.state[ST_SLOT0 + w++] = m.state[ST_SLOT0 + k];
    m.state[ST_SLOT0 + w++] = s;
    m.state[ST_NSLOT] = w;
}

// <e_new, e_slot> for every held slot: grid (n_mol, 8)
__global__ __launch_bounds__(256) void diis_dots_b(const MolDesc* d, int n_mol) {
    const MolDesc& m = d[blockIdx.x];
    const int k = blockIdx.y;
    if (!m.state[ST_ACTIVE] || k >= m.state[ST_NSLOT]) return;
    __shared__ double sh[4];
    const int snew = m.state[ST_SLOT0 + m.state[ST_NSLOT] - 1], sk = m.state[ST_SLOT0 + k];
    const double* x = m.dE[snew];
    const double* y = m.dE[sk];
    const int64_t n = (int64_t)m.N * m.N;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i] * y[i];
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) {
        m.Bmat[snew * 8 + sk] = s;
        m.Bmat[sk * 8 + snew] = s;
    }
}

// Pulay: minimise |sum c_k e_k| with sum c_k = 1 (one thread per molecule);
// with a single vector the coefficient is 1 (no extrapolation).
__global__ void diis_solve_b(const MolDesc* d, int n_mol) {
    const MolDesc& m = d[blockIdx.x];
    if (threadIdx.x != 0 || !m.state[ST_ACTIVE]) return;
    const int ns = m.state[ST_NSLOT];
    if (ns < 2) {
        m.coef[0] = 1.0;
        return;
    }
    double a[9][10];
    const int n = ns + 1;
    for (int i = 0; i < ns; ++i) {
        for (int j = 0; j < ns; ++j) a[i][j] = m.Bmat[m.state[ST_SLOT0 + i] * 8 + m.state[ST_SLOT0 + j]];
        a[i][ns] = -1.0;
        a[i][n] = 0.0;
    }
    for (int j = 0; j < ns; ++j) a[ns][j] = -1.0;
    a[ns][ns] = 0.0;
    a[ns][n] = -1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (piv != c)
            for (int k = 0; k <= n; ++k) { double t = a[c][k]; a[c][k] = a[piv][k]; a[piv][k] = t; }
        double dd = a[c][c] == 0.0 ? 1e-300 : a[c][c];
        for (int r = c + 1; r < n; ++r) {
            double f = a[r][c] / dd;
            for (int k = c; k <= n; ++k) a[r][k] -= f * a[c][k];
        }
    }
    double x[9];
    for (int r = n - 1; r >= 0; --r) {
        double s = a[r][n];
        for (int k = r + 1; k < n; ++k) s -= a[r][k] * x[k];
        x[r] = s / (a[r][r] == 0.0 ? 1e-300 : a[r][r]);
    }
    for (int i = 0; i < ns; ++i) m.coef[i] = x[i];
}

__global__ __launch_bounds__(256) void gersh_b(const MolDesc* d, int n_mol) {
    const MolDesc& m = d[blockIdx.x];
    if (!m.state[ST_ACTIVE]) return;
    __shared__ double sh[4];
    double lo = 1e300, hi = -1e300;
    for (int r = threadIdx.x; r < m.N; r += 256) {
        const double* row = m.T2 + (int64_t)r * m.N;
        double off = 0.0;
        for (int c = 0; c < m.N; ++c)
            if (c != r) off += fabs(row[c]);
        lo = fmin(lo, row[r] - off);
        hi = fmax(hi, row[r] + off);
    }
    lo = -block_max256(-lo, sh);
    hi = block_max256(hi, sh);
    if (threadIdx.x == 0) {
        m.scal[SC_BOUNDS] = lo;
        m.scal[SC_BOUNDS + 1] = hi;
        m.state[ST_TC2] = 1;       // a purification starts
        m.state[ST_TC2U] = 1;
        m.state[ST_TC2X] = -1;
    }
}

// tr X and tr X^2 of a purification step, and when to stop: once
// |tr X - tr X^2| < 1e-11 n_occ, this step's update and one more run (the
// rule of the single-molecule path); later steps of the fixed launch
// sequence find ST_TC2 clear and exit at once.
__global__ __launch_bounds__(256) void traces_b(const MolDesc* d, int n_mol) {
    const MolDesc& m = d[blockIdx.x];
    if (!m.state[ST_ACTIVE]) return;
    if (!m.state[ST_TC2]) {
        if (threadIdx.x == 0) m.state[ST_TC2U] = 0;
        return;
    }
    __shared__ double sh[4];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < m.N; i += 256) {
        a += m.X[(int64_t)i * m.N + i];
        b += m.X2[(int64_t)i * m.N + i];
    }
    a = block_sum256(a, sh);
    b = block_sum256(b, sh);
    if (threadIdx.x == 0) {
        m.scal[SC_TR] = a;
        m.scal[SC_TR + 1] = b;
        m.scal[SC_TR + 2] = a - b;
        m.state[ST_TC2U] = 1;
        int x = m.state[ST_TC2X];
        if (x < 0) {
            if (fabs(a - b) < 1e-11 * (double)max(1, m.n_occ)) x = 1;
        } else if (x > 0) {
            --x;
        }
        if (x == 0) m.state[ST_TC2] = 0;   // this step's update is the last
        m.state[ST_TC2X] = x;
    }
}

// After the purification's fixed launch sequence: a molecule still active
// whose |tr X - tr X^2| never fell below the threshold has no usable
// projector; it is flagged and leaves the batch (later launches skip it).  One
// that reached the threshold but had extra steps left keeps its projector.
__global__ void tc2_check_b(const MolDesc* d, int n_mol) {
    const MolDesc& m = d[blockIdx.x];
    if (threadIdx.x != 0 || !m.state[ST_ACTIVE] || m.state[ST_TC2X] >= 0) return;
    m.state[ST_NOPUR] = 1;
    m.state[ST_ACTIVE] = 0;
    m.state[ST_TC2] = 0;
}

// Cholesky of the n_occ x n_occ (<= 64) Gram matrix Mo and its inverse into
// LinvM (64 x 64, row stride 64), on one wave per molecule.
__global__ __launch_bounds__(64) void small_chol_b(const MolDesc* d, int n_mol) {
    const MolDesc& m = d[blockIdx.x];
    if (!m.state[ST_ACTIVE]) return;
    __shared__ double S[64][65];
    const int lane = threadIdx.x, nb = m.n_occ;
    for (int r = 0; r < 64; ++r)
        S[r][lane] = (r < nb && lane < nb) ? m.Mo[(int64_t)r * nb + lane] : (r == lane ? 1.0 : 0.0);
    __syncthreads();
    int* bad = m.state + ST_BAD;
    double* out = m.LinvM;
    chol_inv64_blocked(S, nb, [&](int) { atomicAdd(bad, 1); }, [&](int i, int c, double v) { out[i * 64 + c] = v; });
}

__global__ void count_active_b(const MolDesc* d, int n_mol, int* out) {
    if (threadIdx.x != 0) return;
    int c = 0;
    for (int i = 0; i < n_mol; ++i) c += d[i].state[ST_ACTIVE];
    *out = c;
}

// -------------------------------------------------- host side
struct Table {
    int* prefix = nullptr;   // device
    int total = 0;
};

struct Plan {
    // purification steps of each launch sequence: tc2_iters inside the
    // captured iteration, tc2_start for the core-Hamiltonian start.  Steps
    // grow with log(spectral width / gap): converged Fock matrices of the
    // 10-60-centre molecules need 27-30, their core Hamiltonians 34-67, and a
    // DIIS-extrapolated Fock matrix of an early iteration can have a smaller
    // gap still (3 of the 256 molecules of the batched workload need more
    // than 64 steps there).  Molecules whose purification has finished skip
    // the remaining steps of the sequence at once.
    int n_mol = 0, prec = 0, tc2_iters = 128, tc2_start = 128;
    bool fin = false;                                     // FP64 exchange once after the FP32 SCF
    MolDesc* d = nullptr;
    Table n2, n2s, rows, pairs, aux, syrk, tail, cq, x[33];   // x[xs], xs = 4 * tiles + quads
    Table x64[33];                                        // FP64 shapes of the final exchange (fin)
    // members on 64 x 64 tiles in t, on 128 x 128 tiles in t128
    struct G { ri::GemmDesc* d = nullptr; Table t, t128; bool ta = false, tb = false; };
    G g_lfx, g_t2, g_x2, g_y, g_mo, g_cp, g_c, g_d, g_fd, g_fds;
    int* n_active = nullptr;
};

#define HC(x)                                  \
    do {                                       \
        hipError_t _e = (x);                   \
        if (_e != hipSuccess) return _e;       \
    } while (0)

hipError_t occupied_space_b(const Plan& p, int tc2_steps, hipStream_t st) {
    const MolDesc* d = p.d;
    const int nm = p.n_mol;
    auto gg = [&](const Plan::G& g) {
        hipError_t e = ri::gemm_grouped(g.ta, g.tb, g.d, g.t.prefix, nm, g.t.total, st, 64);
        return e == hipSuccess ? ri::gemm_grouped(g.ta, g.tb, g.d, g.t128.prefix, nm, g.t128.total, st, 128) : e;
    };
    HC(gg(p.g_lfx));
    HC(gg(p.g_t2));
    gersh_b<<<nm, 256, 0, st>>>(d, nm);
    tc2_init_b<<<p.n2.total, 256, 0, st>>>(d, p.n2.prefix, nm);
    for (int k = 0; k < tc2_steps; ++k) {
        HC(gg(p.g_x2));
        traces_b<<<nm, 256, 0, st>>>(d, nm);
        tc2_update_b<<<p.n2s.total, 256, 0, st>>>(d, p.n2s.prefix, nm);
    }
    tc2_check_b<<<nm, 64, 0, st>>>(d, nm);
    for (int pass = 0; pass < 2; ++pass) {
        HC(gg(p.g_y));
        HC(gg(p.g_mo));
        small_chol_b<<<nm, 64, 0, st>>>(d, nm);
        HC(gg(p.g_cp));
    }
    HC(gg(p.g_c));
    return hipGetLastError();
}

hipError_t iteration_b(const Plan& p, int max_iter, hipStream_t st) {
    const MolDesc* d = p.d;
    const int nm = p.n_mol;
    auto gg = [&](const Plan::G& g) {
        hipError_t e = ri::gemm_grouped(g.ta, g.tb, g.d, g.t.prefix, nm, g.t.total, st, 64);
        return e == hipSuccess ? ri::gemm_grouped(g.ta, g.tb, g.d, g.t128.prefix, nm, g.t128.total, st, 128) : e;
    };
    // Fock build
    HC(ri::zero_tail_b(d, p.tail.prefix, nm, p.tail.total, p.prec, st));
    HC(ri::gamma_j_b(d, nm, p.pairs.prefix, p.pairs.total, p.aux.prefix, p.aux.total, p.n2.prefix, p.n2.total, st));
    HC(ri::cpad_b(d, p.cq.prefix, nm, p.cq.total, p.prec, st));
    for (int xs = 1; xs <= 32; ++xs)
        if (p.x[xs].total > 0) HC(ri::x_transform_b(d, p.x[xs].prefix, nm, p.x[xs].total, xs, p.prec, st));
    HC(ri::syrk_b(d, p.syrk.prefix, nm, p.syrk.total, p.prec, st));
    HC(ri::kreduce_b(d, p.rows.prefix, nm, p.rows.total, st));
    // F, D, energy, error, convergence
    fock_assemble_b<<<p.n2.total, 256, 0, st>>>(d, p.n2.prefix, nm);
    HC(gg(p.g_d));
    HC(gg(p.g_fd));
    HC(gg(p.g_fds));
    commutator_b<<<p.n2.total, 256, 0, st>>>(d, p.n2.prefix, nm);
    energy_conv_b<<<nm, 256, 0, st>>>(d, nm, max_iter);
    // DIIS and the next occupied space (molecules that just converged skip)
    diis_push_b<<<p.n2.total, 256, 0, st>>>(d, p.n2.prefix, nm);
    diis_book_b<<<nm, 64, 0, st>>>(d, nm);
    diis_dots_b<<<dim3(nm, 8), 256, 0, st>>>(d, nm);
    diis_solve_b<<<nm, 64, 0, st>>>(d, nm);
    diis_combine_b<<<p.n2.total, 256, 0, st>>>(d, p.n2.prefix, nm);
    HC(occupied_space_b(p, p.tc2_iters, st));
    count_active_b<<<1, 64, 0, st>>>(d, nm, p.n_active);
    return hipGetLastError();
}


// The final FP64 exchange of an FP32 SCF.  The descriptors carry xs = xs64
// (uploaded in place of the FP32 ones); the Fock build's exchange launches
// then run in FP64 arithmetic on the FP32-stored B and the orbitals C of the
// last iteration.
hipError_t final_fp64_b(const Plan& p, hipStream_t st) {
    const MolDesc* d = p.d;
    const int nm = p.n_mol;
    final_begin_b<<<nm, 64, 0, st>>>(d, nm);
    HC(hipGetLastError());
    HC(ri::zero_tail_b(d, p.tail.prefix, nm, p.tail.total, RI_FP64, st));
    HC(ri::cpad_b(d, p.cq.prefix, nm, p.cq.total, RI_FP64, st));
    for (int xs = 1; xs <= 32; ++xs)
        if (p.x64[xs].total > 0)
            HC(ri::x_transform_b(d, p.x64[xs].prefix, nm, p.x64[xs].total, xs, ri::X_F64_B32, st));
    HC(ri::syrk_b(d, p.syrk.prefix, nm, p.syrk.total, RI_FP64, st));
    HC(ri::kreduce_b(d, p.rows.prefix, nm, p.rows.total, st));
    energy_final_b<<<nm, 256, 0, st>>>(d, nm);
    return hipGetLastError();
}

}  // namespace

namespace {

struct Carver {
    char* base;
    size_t cap, off = 0;
    template <class T>
    T* take(int64_t n) {
        size_t b = ((size_t)(n < 0 ? 0 : n) * sizeof(T) + 255) & ~(size_t)255;
        size_t o = off;
        off += b;
        return base ? (T*)(base + o) : nullptr;
    }
};

int k_split_small(int64_t rows) { return (int)std::max<int64_t>(1, std::min<int64_t>(8, rows / 16384)); }

// Lays out (or, with base == nullptr, sizes) the batch workspace and fills
// the host copies of the descriptors and tables.
struct HostPlan {
    std::vector<MolDesc> mols;
    std::vector<int> tile;                            // GEMM tile edge per molecule
    std::vector<Table*> tabs;                         // every table, in layout order
    std::vector<std::vector<int>> prefixes;           // each table's prefix (same order)
    std::vector<Plan::G*> gs;                         // every grouped GEMM
    std::vector<std::vector<ri::GemmDesc>> gemms;     // each grouped GEMM's members (same order)
};

int tune_bucket(int N, int n_buckets) { return std::min((N + 127) / 128, n_buckets) - 1; }

// Tiles of an M x N product on tile x tile tiles (upper ones only for a
// symmetric product).
int gemm_tiles(int M, int N, int tile, bool sym) {
    const int tm = (M + tile - 1) / tile, tn = (N + tile - 1) / tile;
    return sym ? tn * (tn + 1) / 2 : tm * tn;
}

bool tuning_ok(const ri_batch_tuning* t) {
    if (!t) return true;
    if (t->n_buckets < 1 || t->n_buckets > RI_TUNE_BUCKETS) return false;
    for (int b = 0; b < t->n_buckets; ++b)
        if ((t->gemm_tile[b] != 64 && t->gemm_tile[b] != 128) || t->syrk_split[b] < 1 || t->syrk_split[b] > RI_TUNE_MAX_SPLIT)
            return false;
    return true;
}

// SYRK split of a molecule's reduction length into ks pieces of a multiple of 16 rows
void set_split(MolDesc& m, int ks) {
    m.ks = ks;
    m.chunk = ((m.rows_pad + m.ks - 1) / m.ks + 15) / 16 * 16;
    m.ks = (int)((m.rows_pad + m.chunk - 1) / m.chunk);
}

}  // namespace

// The workspace layout shared by the size query and the solver.
static int32_t batch_layout(int32_t n_mol, const ri_system* sys, const ri_batch_mol* mol, int32_t prec, int diis_n,
                            const ri_batch_tuning* tune, Carver& cv, Plan& p, HostPlan& hp) {
    p.n_mol = n_mol;
    p.fin = (prec & RI_FINAL_FP64) != 0;
    prec &= ~RI_FINAL_FP64;
    p.prec = prec;
    const bool wide = prec == RI_FP64 || p.fin;   // Xt and Cq hold FP64 at some point
    hp.mols.assign(n_mol, MolDesc{});
    hp.tile.assign(n_mol, 64);
    for (int i = 0; i < n_mol; ++i) {
        const ri_system& s = sys[i];
        MolDesc& m = hp.mols[i];
        const int N = s.n_fn, na = s.n_aux, no = s.n_occ;
        if (N <= 0 || na <= 0 || no <= 0 || no > 64 || no > N) return RI_E_UNSUPPORTED;
        m.N = N; m.n_aux = na; m.n_occ = no; m.diis_n = diis_n;
        m.nt = ri::n_tiles_1d(N);
        m.npad = ri::xt_ld(N);
        m.ntl = ri::n_tiles(N);
        m.n_pairs = mol[i].n_pairs;
        {
            // FP64: whole 16-row tiles, and 4-row quads in place of a last tile of 12 rows or
            // fewer; FP32: whole tiles only
            const int mt = (no + 15) / 16, rem = no - 16 * (mt - 1);
            m.xs64 = rem <= 12 ? 4 * (mt - 1) + (rem + 3) / 4 : 4 * mt;
            m.xs = prec == RI_FP64 ? m.xs64 : 4 * mt;
        }
        const int64_t rows = (int64_t)na * no;
        m.rows_pad = (rows + 15) / 16 * 16;
        if (tune) {
            const int b = tune_bucket(N, tune->n_buckets);
            set_split(m, tune->syrk_split[b]);
            hp.tile[i] = tune->gemm_tile[b];
        } else {
            set_split(m, k_split_small(rows));
        }
        m.pairs = mol[i].pairs;
        m.Bc = mol[i].Bc;
        m.B = mol[i].B;
        m.C = mol[i].C_occ;
        const int64_t n2 = (int64_t)N * N;
        m.J = cv.take<double>(n2); m.K = cv.take<double>(n2); m.gamma = cv.take<double>(na);
        m.dpair = cv.take<double>(std::max<int64_t>(1, m.n_pairs));
        m.part = cv.take<double>((int64_t)RI_TUNE_MAX_SPLIT * m.npad * m.npad);   // the largest split any tuning may choose
        m.Xt = cv.take<char>((m.rows_pad + 16) * m.npad * (wide ? 8 : 4));
        double** mats[] = {&m.S, &m.H, &m.LinvS, &m.F, &m.D, &m.T1, &m.T2, &m.E, &m.Fx, &m.X, &m.X2};
        for (double** q : mats) *q = cv.take<double>(n2);
        for (int k = 0; k < 8; ++k) {
            m.dF[k] = k < diis_n ? cv.take<double>(n2) : nullptr;
            m.dE[k] = k < diis_n ? cv.take<double>(n2) : nullptr;
        }
        m.Y = cv.take<double>((int64_t)N * no);
        m.Cp = cv.take<double>((int64_t)N * no);
        // padded C for the X launch: FP64 [64 nt][64] doubles, FP32 the same shape in floats
        m.Cq = cv.take<double>((int64_t)m.nt * 64 * (wide ? 64 : 32));
        m.Mo = cv.take<double>((int64_t)no * no);
        m.LinvM = cv.take<double>(64 * 64);
        m.dinvM = cv.take<double>(((N + 63) / 64) * 4096);   // Cholesky diagonal blocks of S
        m.Bmat = cv.take<double>(64);
        m.coef = cv.take<double>(8);
        m.scal = cv.take<double>(32);
        m.state = cv.take<int>(ST_N);
    }
    // tables
    auto mk = [&](std::vector<int> counts, Table& t) {
        std::vector<int> pre(n_mol + 1, 0);
        for (int i = 0; i < n_mol; ++i) pre[i + 1] = pre[i] + counts[i];
        t.total = pre[n_mol];
        t.prefix = cv.take<int>(n_mol + 1);
        hp.tabs.push_back(&t);
        hp.prefixes.push_back(pre);
    };
    std::vector<int> c(n_mol);
    for (int i = 0; i < n_mol; ++i) c[i] = (int)(((int64_t)hp.mols[i].N * hp.mols[i].N + 255) / 256);
    mk(c, p.n2);
    for (int i = 0; i < n_mol; ++i) c[i] = (int)(((int64_t)hp.mols[i].N * hp.mols[i].N + 2047) / 2048);
    mk(c, p.n2s);
    for (int i = 0; i < n_mol; ++i) c[i] = hp.mols[i].N;
    mk(c, p.rows);
    for (int i = 0; i < n_mol; ++i) c[i] = (int)((hp.mols[i].n_pairs + 255) / 256);
    mk(c, p.pairs);
    for (int i = 0; i < n_mol; ++i) c[i] = hp.mols[i].n_aux;
    mk(c, p.aux);
    for (int i = 0; i < n_mol; ++i) {
        const int t128 = hp.mols[i].npad / 128;
        c[i] = t128 * (t128 + 1) / 2 * hp.mols[i].ks;
    }
    mk(c, p.syrk);
    for (int i = 0; i < n_mol; ++i) c[i] = 16;
    mk(c, p.tail);
    for (int i = 0; i < n_mol; ++i) c[i] = hp.mols[i].nt;
    mk(c, p.cq);
    for (int xs = 1; xs <= 32; ++xs) {
        for (int i = 0; i < n_mol; ++i)
            c[i] = hp.mols[i].xs == xs ? hp.mols[i].nt * ((hp.mols[i].n_aux + 1) / 2) : 0;
        mk(c, p.x[xs]);
    }
    if (p.fin)
        for (int xs = 1; xs <= 32; ++xs) {
            for (int i = 0; i < n_mol; ++i)
                c[i] = hp.mols[i].xs64 == xs ? hp.mols[i].nt * ((hp.mols[i].n_aux + 1) / 2) : 0;
            mk(c, p.x64[xs]);
        }
    // grouped GEMMs: member i of each
    // tunable: the member runs on the molecule's tuned tile (else on 64 x 64)
    auto mkg = [&](Plan::G& g, bool ta, bool tb, bool tunable, auto fill, int act = ST_ACTIVE, bool sym = false) {
        g.ta = ta;
        g.tb = tb;
        std::vector<ri::GemmDesc> v(n_mol);
        std::vector<int> c64(n_mol), c128(n_mol);
        for (int i = 0; i < n_mol; ++i) {
            fill(hp.mols[i], v[i]);
            v[i].sym = sym;
            // runs while this flag is set (no pointer in the sizing pass, whose carver has no base)
            v[i].active = hp.mols[i].state ? hp.mols[i].state + act : nullptr;
            const bool big = tunable && hp.tile[i] == 128;
            c64[i] = big ? 0 : gemm_tiles(v[i].M, v[i].N, 64, sym);
            c128[i] = big ? gemm_tiles(v[i].M, v[i].N, 128, sym) : 0;
        }
        g.d = cv.take<ri::GemmDesc>(n_mol);
        hp.gs.push_back(&g);
        hp.gemms.push_back(v);
        mk(c64, g.t);
        mk(c128, g.t128);
    };
    auto set = [](ri::GemmDesc& g, int M, int N, int K, double al, const double* A, int64_t lda, const double* B,
                  int64_t ldb, double* C, int64_t ldc, int tri) {
        g.M = M; g.N = N; g.K = K; g.tri = tri; g.alpha = al; g.beta = 0.0;
        g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc; g.sym = 0;
    };
    mkg(p.g_lfx, false, false, true, [&](MolDesc& m, ri::GemmDesc& g) { set(g, m.N, m.N, m.N, 1.0, m.LinvS, m.N, m.Fx, m.N, m.T1, m.N, 1); });
    // L_S^{-1} Fx L_S^{-T} and 2 C C^T are symmetric: upper tiles only, mirrored
    mkg(p.g_t2, false, true, true, [&](MolDesc& m, ri::GemmDesc& g) { set(g, m.N, m.N, m.N, 1.0, m.T1, m.N, m.LinvS, m.N, m.T2, m.N, 0); },
        ST_ACTIVE, true);
    // the purification square X X of a symmetric X: upper tiles only, mirrored
    mkg(p.g_x2, false, false, true, [&](MolDesc& m, ri::GemmDesc& g) { set(g, m.N, m.N, m.N, 1.0, m.X, m.N, m.X, m.N, m.X2, m.N, 0); },
        ST_TC2, true);
    mkg(p.g_y, false, false, false, [&](MolDesc& m, ri::GemmDesc& g) { set(g, m.N, m.n_occ, m.N, 1.0, m.X, m.N, m.Cp, m.n_occ, m.Y, m.n_occ, 0); });
    mkg(p.g_mo, true, false, false, [&](MolDesc& m, ri::GemmDesc& g) { set(g, m.n_occ, m.n_occ, m.N, 1.0, m.Y, m.n_occ, m.Y, m.n_occ, m.Mo, m.n_occ, 0); });
    mkg(p.g_cp, false, true, false, [&](MolDesc& m, ri::GemmDesc& g) { set(g, m.N, m.n_occ, m.n_occ, 1.0, m.Y, m.n_occ, m.LinvM, 64, m.Cp, m.n_occ, 0); });
    mkg(p.g_c, true, false, false, [&](MolDesc& m, ri::GemmDesc& g) { set(g, m.N, m.n_occ, m.N, 1.0, m.LinvS, m.N, m.Cp, m.n_occ, m.C, m.n_occ, 2); });
    mkg(p.g_d, false, true, false, [&](MolDesc& m, ri::GemmDesc& g) { set(g, m.N, m.N, m.n_occ, 2.0, m.C, m.n_occ, m.C, m.n_occ, m.D, m.N, 0); },
        ST_ACTIVE, true);
    mkg(p.g_fd, false, false, true, [&](MolDesc& m, ri::GemmDesc& g) { set(g, m.N, m.N, m.N, 1.0, m.F, m.N, m.D, m.N, m.T1, m.N, 0); });
    mkg(p.g_fds, false, false, true, [&](MolDesc& m, ri::GemmDesc& g) { set(g, m.N, m.N, m.N, 1.0, m.T1, m.N, m.S, m.N, m.T2, m.N, 0); });
    p.d = cv.take<MolDesc>(n_mol);
    p.n_active = cv.take<int>(4);
    return RI_OK;
}

namespace {

#define HIPR(x)                                                          \
    do {                                                                 \
        hipError_t _e = (x);                                             \
        if (_e != hipSuccess) { ri::set_hip_error(hipGetErrorString(_e)); return RI_E_HIP; } \
    } while (0)

int32_t check_batch(int32_t n_mol, const ri_system* sys, const ri_batch_mol* mol, int32_t prec) {
    if (n_mol <= 0 || !sys || !mol) return RI_E_ARG;
    if (prec != RI_FP64 && prec != RI_FP32 && prec != (RI_FP32 | RI_FINAL_FP64)) return RI_E_UNSUPPORTED;
    for (int i = 0; i < n_mol; ++i) {
        const ri_system& s = sys[i];
        if (s.n_centres <= 0 || s.n_fn <= 0 || s.n_aux <= 0 || s.n_occ <= 0 || !s.xyz || !s.Z || !s.fn_centre ||
            !s.fn_exp || !s.aux_centre || !s.aux_exp || !mol[i].B || !mol[i].C_occ || mol[i].n_pairs < 0 ||
            (mol[i].n_pairs > 0 && (!mol[i].Bc || !mol[i].pairs)))
            return RI_E_ARG;
    }
    return RI_OK;
}

int32_t upload_plan(const Plan& p, const HostPlan& hp, hipStream_t st) {
    const int n_mol = p.n_mol;
    HIPR(hipMemcpyAsync(p.d, hp.mols.data(), sizeof(MolDesc) * n_mol, hipMemcpyHostToDevice, st));
    for (size_t k = 0; k < hp.tabs.size(); ++k)
        HIPR(hipMemcpyAsync(hp.tabs[k]->prefix, hp.prefixes[k].data(), sizeof(int) * (n_mol + 1),
                            hipMemcpyHostToDevice, st));
    for (size_t k = 0; k < hp.gs.size(); ++k)
        HIPR(hipMemcpyAsync(hp.gs[k]->d, hp.gemms[k].data(), sizeof(ri::GemmDesc) * n_mol, hipMemcpyHostToDevice,
                            st));
    HIPR(hipStreamSynchronize(st));   // host vectors are read by the copies above
    return RI_OK;
}

// Mean time in ms of `reps` launches of fn after one untimed launch.
template <class F>
int32_t time_ms(F fn, hipStream_t st, hipEvent_t e0, hipEvent_t e1, int reps, float* ms) {
    HIPR(fn());
    HIPR(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) HIPR(fn());
    HIPR(hipEventRecord(e1, st));
    HIPR(hipEventSynchronize(e1));
    float t = 0.f;
    HIPR(hipEventElapsedTime(&t, e0, e1));
    *ms = t / reps;
    return RI_OK;
}

int32_t autotune_impl(int32_t n_mol, const ri_system* sys, const ri_batch_mol* mol, int32_t prec,
                      ri_batch_tuning* out, void* ws, size_t ws_bytes, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    Carver cv{(char*)ws, ws_bytes};
    Plan p;
    HostPlan hp;
    int32_t rc = batch_layout(n_mol, sys, mol, prec, 8, nullptr, cv, p, hp);
    if (rc != RI_OK) return rc;
    if (cv.off + 256 > ws_bytes) return RI_E_WORKSPACE;
    rc = upload_plan(p, hp, st);
    if (rc != RI_OK) return rc;
    // every molecule active; operands zeroed (the timings do not depend on values)
    state_init_b<<<n_mol, 256, 0, st>>>(p.d, n_mol);
    HIPR(hipGetLastError());
    for (const MolDesc& m : hp.mols) {
        HIPR(ri::fill(m.X, 0.0, (int64_t)m.N * m.N, st));
        const int64_t xt = (m.rows_pad + 16) * m.npad * ((prec & ~RI_FINAL_FP64) == RI_FP64 || p.fin ? 8 : 4);
        HIPR(ri::fill((double*)m.Xt, 0.0, xt / 8, st));
    }
    std::memset(out, 0, sizeof(*out));
    int nb = 1;
    for (const MolDesc& m : hp.mols) nb = std::max(nb, tune_bucket(m.N, RI_TUNE_BUCKETS) + 1);
    out->n_buckets = nb;
    Plan::G& gx = p.g_x2;
    for (int b = 0; b < nb; ++b) {
        std::vector<int> members;
        for (int i = 0; i < n_mol; ++i)
            if (tune_bucket(hp.mols[i].N, RI_TUNE_BUCKETS) == b) members.push_back(i);
        out->gemm_tile[b] = 64;
        out->syrk_split[b] = 1;
        if (members.empty()) continue;
        // GEMM tile: the purification square X X of the bucket's molecules
        float best = 1e30f;
        for (int tile : {64, 128}) {
            std::vector<int> pre(n_mol + 1, 0);
            for (int i = 0; i < n_mol; ++i) {
                const int M = hp.mols[i].N;
                const int t = gemm_tiles(M, M, tile, true);
                pre[i + 1] = pre[i] + (tune_bucket(M, RI_TUNE_BUCKETS) == b ? t : 0);
            }
            HIPR(hipMemcpyAsync(gx.t.prefix, pre.data(), sizeof(int) * (n_mol + 1), hipMemcpyHostToDevice, st));
            float ms = 0.f;
            rc = time_ms([&] { return ri::gemm_grouped(gx.ta, gx.tb, gx.d, gx.t.prefix, n_mol, pre[n_mol], st, tile); },
                         st, e0, e1, 2, &ms);
            if (rc != RI_OK) return rc;
            if (ms < best) { best = ms; out->gemm_tile[b] = tile; out->gemm_ms[b] = ms; }
        }
        // SYRK split: SYRK partials and their reduction for the bucket's molecules;
        // candidates from the widest down (time grows as the split narrows),
        // stopping once one is 1.1x the best
        best = 1e30f;
        for (int ks : {16, 8, 4, 2, 1}) {
            std::vector<int> ps(n_mol + 1, 0), pr(n_mol + 1, 0);
            std::vector<MolDesc> mols = hp.mols;
            for (int i = 0; i < n_mol; ++i) {
                const bool in = tune_bucket(mols[i].N, RI_TUNE_BUCKETS) == b;
                if (in) set_split(mols[i], ks);
                const int t128 = mols[i].npad / 128;
                ps[i + 1] = ps[i] + (in ? t128 * (t128 + 1) / 2 * mols[i].ks : 0);
                pr[i + 1] = pr[i] + (in ? mols[i].N : 0);
            }
            HIPR(hipMemcpyAsync(p.d, mols.data(), sizeof(MolDesc) * n_mol, hipMemcpyHostToDevice, st));
            HIPR(hipMemcpyAsync(p.syrk.prefix, ps.data(), sizeof(int) * (n_mol + 1), hipMemcpyHostToDevice, st));
            HIPR(hipMemcpyAsync(p.rows.prefix, pr.data(), sizeof(int) * (n_mol + 1), hipMemcpyHostToDevice, st));
            float ms = 0.f;
            rc = time_ms([&] {
                hipError_t e = ri::syrk_b(p.d, p.syrk.prefix, n_mol, ps[n_mol], p.prec, st);
                return e == hipSuccess ? ri::kreduce_b(p.d, p.rows.prefix, n_mol, pr[n_mol], st) : e;
            }, st, e0, e1, 2, &ms);
            if (rc != RI_OK) return rc;   // the host vectors stay alive until the timing synchronised
            if (ms < best) { best = ms; out->syrk_split[b] = ks; out->syrk_ms[b] = ms; }
            if (ms > 1.1f * best) break;
        }
    }
    HIPR(hipStreamSynchronize(st));
    return RI_OK;
}

}  // namespace

extern "C" {

size_t ri_energy_batched_workspace(int32_t n_mol, const ri_system* sys, const ri_batch_mol* mol, int32_t prec) {
    if (n_mol <= 0 || !sys || !mol || check_batch(n_mol, sys, mol, prec) == RI_E_UNSUPPORTED) return 0;
    Carver cv{nullptr, 0};
    Plan p;
    HostPlan hp;
    if (batch_layout(n_mol, sys, mol, prec, 8, nullptr, cv, p, hp) != RI_OK) return 0;
    return cv.off + 256;
}

int32_t ri_batch_autotune(int32_t n_mol, const ri_system* sys, const ri_batch_mol* mol, int32_t prec,
                          ri_batch_tuning* out, void* ws, size_t ws_bytes, hipStream_t st) {
    if (!out || !ws) return RI_E_ARG;
    int32_t rc = check_batch(n_mol, sys, mol, prec);
    if (rc != RI_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPR(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        ri::set_hip_error("hipEventCreate failed");
        return RI_E_HIP;
    }
    rc = autotune_impl(n_mol, sys, mol, prec, out, ws, ws_bytes, st, e0, e1);
    if (rc == RI_E_HIP) hipStreamSynchronize(st);   // let queued copies read their host sources
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rc;
}

int32_t ri_energy_batched(int32_t n_mol, const ri_system* sys, const ri_batch_mol* mol, int32_t prec,
                          const ri_scf_opts* opts, int32_t use_graph, const ri_batch_tuning* tuning,
                          ri_scf_result* res, void* ws, size_t ws_bytes, hipStream_t st) {
    if (!opts || !res || !ws || !tuning_ok(tuning)) return RI_E_ARG;
    int32_t rc = check_batch(n_mol, sys, mol, prec);
    if (rc != RI_OK) return rc;
    if (opts->diis_n < 1 || opts->diis_n > 8 || opts->max_iter < 1 || !(opts->tol_E > 0) || !(opts->tol_err > 0) ||
        opts->guess_kind != 0 || opts->max_purify < 0)
        return RI_E_ARG;
    Carver cv{(char*)ws, ws_bytes};
    Plan p;
    HostPlan hp;
    rc = batch_layout(n_mol, sys, mol, prec, 8, tuning, cv, p, hp);
    if (rc != RI_OK) return rc;
    if (cv.off + 256 > ws_bytes) return RI_E_WORKSPACE;
    for (auto& m : hp.mols) {
        m.tol_E = opts->tol_E;
        m.tol_err = opts->tol_err;
        m.diis_n = opts->diis_n;
    }
    if (opts->max_purify > 0) p.tc2_iters = p.tc2_start = opts->max_purify;
    rc = upload_plan(p, hp, st);
    if (rc != RI_OK) return rc;
    // per-molecule setup: S, h, E_nn, Cholesky of S and L_S^{-1}.  Each
    // molecule's chain is a series of small launches on its own buffers, so
    // the molecules are spread over SETUP_STREAMS streams forked from and
    // joined back into `st` (a non-positive pivot is reported by atomicMin)
    constexpr int SETUP_STREAMS = 4;
    // On every exit the caller's stream waits for all of them before they are
    // destroyed, so no setup work is left running after an error return.
    struct SetupStreams {
        hipStream_t st;
        hipStream_t s[SETUP_STREAMS] = {};
        hipEvent_t e[SETUP_STREAMS + 1] = {};
        ~SetupStreams() {
            for (int k = 0; k < SETUP_STREAMS; ++k) {
                if (!s[k]) continue;
                hipEvent_t j = nullptr;
                if (hipEventCreateWithFlags(&j, hipEventDisableTiming) == hipSuccess) {
                    if (hipEventRecord(j, s[k]) == hipSuccess) (void)hipStreamWaitEvent(st, j, 0);
                    (void)hipEventDestroy(j);
                } else {
                    (void)hipStreamSynchronize(s[k]);
                }
            }
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
            for (hipStream_t x : s)
                if (x) (void)hipStreamDestroy(x);
        }
    } ss{st};
    int* bad = p.n_active + 1;
    HIPR(ri::fill_i32(bad, INT_MAX, 1, st));
    HIPR(hipEventCreateWithFlags(&ss.e[SETUP_STREAMS], hipEventDisableTiming));
    HIPR(hipEventRecord(ss.e[SETUP_STREAMS], st));
    for (int k = 0; k < SETUP_STREAMS; ++k) {
        HIPR(hipStreamCreateWithFlags(&ss.s[k], hipStreamNonBlocking));
        HIPR(hipEventCreateWithFlags(&ss.e[k], hipEventDisableTiming));
        HIPR(hipStreamWaitEvent(ss.s[k], ss.e[SETUP_STREAMS], 0));
    }
    for (int i = 0; i < n_mol; ++i) {
        const MolDesc& m = hp.mols[i];
        hipStream_t si = ss.s[i % SETUP_STREAMS];
        HIPR(ri::one_electron(&sys[i], m.S, m.H, si));
        HIPR(ri::nuclear_repulsion(&sys[i], m.scal + SC_ENUC, si));
        HIPR(ri::copy(m.T1, m.S, (int64_t)m.N * m.N, si));
        HIPR(ri::cholesky_inv(m.T1, m.N, m.N, m.LinvS, m.N, m.dinvM, bad, si));
    }
    for (int k = 0; k < SETUP_STREAMS; ++k) {
        HIPR(hipEventRecord(ss.e[k], ss.s[k]));
        HIPR(hipStreamWaitEvent(st, ss.e[k], 0));
    }
    state_init_b<<<n_mol, 256, 0, st>>>(p.d, n_mol);
    hash_cp_b<<<n_mol, 256, 0, st>>>(p.d, n_mol);
    HIPR(hipGetLastError());
    int hbad = INT_MAX;
    HIPR(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPR(hipStreamSynchronize(st));
    if (hbad != INT_MAX) return RI_E_NOT_PD;
    // core-Hamiltonian start
    copy_h_b<<<p.n2.total, 256, 0, st>>>(p.d, p.n2.prefix, n_mol);
    HIPR(occupied_space_b(p, p.tc2_start, st));
    // iterations.  A graph is captured on a private non-blocking stream (the
    // caller's stream may be the legacy default stream, which cannot be
    // captured); the host waits for every iteration, so ordering with the
    // caller's stream is kept by synchronising before the first replay.
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cs = st;
    if (use_graph) {
        HIPR(hipStreamSynchronize(st));
        HIPR(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e0 = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        hipError_t e = e0 == hipSuccess ? iteration_b(p, opts->max_iter, cs) : e0;
        hipError_t e2 = e0 == hipSuccess ? hipStreamEndCapture(cs, &graph) : hipSuccess;
        hipError_t e3 = (e == hipSuccess && e2 == hipSuccess) ? hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)
                                                               : hipSuccess;
        if (e != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            hipStreamDestroy(cs);
            HIPR(e != hipSuccess ? e : (e2 != hipSuccess ? e2 : e3));
        }
    }
    int active = n_mol;
    hipError_t loop_err = hipSuccess;
    for (int it = 0; it < opts->max_iter && active > 0; ++it) {
        loop_err = use_graph ? hipGraphLaunch(exec, cs) : iteration_b(p, opts->max_iter, cs);
        if (loop_err == hipSuccess) loop_err = hipMemcpyAsync(&active, p.n_active, sizeof(int), hipMemcpyDeviceToHost, cs);
        if (loop_err == hipSuccess) loop_err = hipStreamSynchronize(cs);
        if (loop_err != hipSuccess) break;
    }
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (cs != st) hipStreamDestroy(cs);
    HIPR(loop_err);
    if (p.fin) {
        std::vector<MolDesc> d64 = hp.mols;
        for (MolDesc& m : d64) m.xs = m.xs64;
        HIPR(hipMemcpyAsync(p.d, d64.data(), sizeof(MolDesc) * n_mol, hipMemcpyHostToDevice, st));
        HIPR(hipStreamSynchronize(st));   // d64 is read by the copy
        HIPR(final_fp64_b(p, st));
    }
    // results
    bool all = true, nopur = false;
    for (int i = 0; i < n_mol; ++i) {
        const MolDesc& m = hp.mols[i];
        double sc[8];
        int stt[ST_N];
        HIPR(hipMemcpyAsync(sc, m.scal, sizeof(sc), hipMemcpyDeviceToHost, st));
        HIPR(hipMemcpyAsync(stt, m.state, sizeof(stt), hipMemcpyDeviceToHost, st));
        HIPR(hipStreamSynchronize(st));
        ri_scf_result& r = res[i];
        r.E_total = sc[0]; r.E_nuc = sc[1]; r.E_1e = sc[2]; r.E_J = sc[3]; r.E_K = sc[4];
        r.max_err = sc[5]; r.last_dE = sc[7];
        r.n_iter = stt[ST_IT];
        r.converged = stt[ST_CONV];
        all = all && stt[ST_CONV];
        nopur = nopur || stt[ST_NOPUR];
        if (mol[i].F) HIPR(ri::copy(mol[i].F, m.F, (int64_t)m.N * m.N, st));
    }
    HIPR(hipStreamSynchronize(st));
    return nopur ? RI_E_NO_PURIFY : (all ? RI_OK : RI_E_NO_CONV);
}

}  // extern "C"
