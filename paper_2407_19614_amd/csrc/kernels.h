// Launchers of the method's kernels (integrals, Fock build, SCF, gradient).
#pragma once
#include "common.h"

#include <functional>

namespace ri {

// Band of the factor for the solve's leaves: 4 ceil(n/64) slots of 4096
// doubles (Dinv_k and -L_{k+d,k}, d = 1..3, in MFMA operand order), from the
// factor L and the diagonal-block inverses Dinv left by cholesky_inv.
hipError_t trsm_band(const double* L, int n, int64_t lda, const double* Dinv, double* P, hipStream_t s);

// Recursive in-place B <- L^{-1} B (see gemm.hip) with P from trsm_band;
// done(r0, r1) runs in stream order once rows r0 .. r1 of B are final (r0
// offsets the row numbers).
hipError_t trsm_rec(const double* L, int n, int64_t lda, const double* P, double* B, int ncols, int64_t ldb,
                    hipStream_t s, int r0, const std::function<hipError_t(int, int)>& done);

// ---- integrals
hipError_t screen_pairs(const ri_system* s, double tau, int32_t* counts, int64_t* offsets, hipStream_t st);
hipError_t write_pairs(const ri_system* s, double tau, const int64_t* offsets, int32_t* pairs, hipStream_t st);
hipError_t eri3(const ri_system* s, const int32_t* pairs, int64_t n_pairs, double* T, hipStream_t st);
hipError_t metric(const ri_system* s, double* A, hipStream_t st);
hipError_t one_electron(const ri_system* s, double* S, double* H, hipStream_t st);
hipError_t nuclear_repulsion(const ri_system* s, double* out, hipStream_t st);

// ---- packed B geometry
inline int n_tiles_1d(int N) { return (N + 63) / 64; }
inline int64_t n_tiles(int N) { int t = n_tiles_1d(N); return (int64_t)t * (t + 1) / 2; }
inline int64_t tile_elems(int N) { return n_tiles(N) * 4096; }

hipError_t pair_map(const int32_t* pairs, int64_t n_pairs, int N, int32_t* map, hipStream_t st);
hipError_t pack_b(const double* Bc, int64_t n_pairs, const int32_t* map, int N, int n_aux, void* B,
                  int prec, hipStream_t st);

// ---- Fock build pieces
// Xt[P][i][mu] (row stride Npad = 64 * tiles) = (B^P C_occ)^T
// Cp: workspace for C_occ zero-padded to [64 * tiles][cpad_ld(n_occ)].
// prec RI_FP64, RI_FP32, or X_F64_B32: FP64 arithmetic (FP64 Cp and Xt) on
// FP32-stored B, widened exactly on load.
constexpr int X_F64_B32 = 0x41;
int cpad_ld(int n_occ);
int64_t cpad_elems(int N, int n_occ);
hipError_t x_transform(const void* B, int prec, int N, int n_aux, int n_occ, const double* C,
                       double* Cp, void* Xt, hipStream_t st);
// K = sum_P X^P X^P^T from Xt; part = workspace of n_split * Npad^2 doubles.
hipError_t k_syrk(const void* Xt, int prec, int N, int n_aux, int n_occ, double* part, int n_split,
                  double* K, hipStream_t st);
int k_split_count(int N, int n_aux, int n_occ);
int64_t xt_rows(int n_aux, int n_occ);
int xt_ld(int N);
// gamma and J from the compressed FP64 tensor.
// gamma and J from pair weights dpair (w D_mu_nu, w = 1 on the diagonal, 2 off it).
// cap > 0 limits the gamma and J-partial launches to cap workgroups each (grid-stride;
// same results), so they can run beside the exchange kernels on a side stream.
hipError_t gamma_j_pairs(const double* Bc, const int32_t* pairs, int64_t n_pairs, int N, int n_aux,
                         const double* dpair, double* gamma, double* jpart, int n_jsplit, double* J, hipStream_t st,
                         int cap = 0);
// pair weights of a density matrix D [N][N] (symmetrised)
hipError_t dpair_density(const int32_t* pairs, int64_t n_pairs, const double* D, int N, double* dpair, hipStream_t st);
// K = 1/2 sum_P B^P D B^P from B_c, slab of S auxiliaries at a time (workspace map [N*N],
// Bf [S][N][N], Y [N][S*N]); K symmetrised.
hipError_t k_density(const double* Bc, const int32_t* pairs, int64_t n_pairs, int N, int n_aux, const double* D,
                     int32_t* map, double* Bf, double* Y, int S, double* K, hipStream_t st);
hipError_t gamma_j(const double* Bc, const int32_t* pairs, int64_t n_pairs, int N, int n_aux,
                   int n_occ, const double* C, double* dpair, double* gamma, double* jpart,
                   int n_jsplit, double* J, hipStream_t st, int cap = 0);
// Workgroups of each gamma / J launch beside an FP64 or FP32 exchange, applied when
// B_c has at least GJ_SIDE_MIN elements (N = 1000: 2e8; there 64 workgroups made
// gamma / J the critical path and 256 slowed X on every CU).
constexpr int GJ_SIDE_CAP = 128;
constexpr int64_t GJ_SIDE_MIN = 100000000;
int j_split_count(int n_aux);

}  // namespace ri

namespace ri {
// ---- SCF helpers (scf.hip)
hipError_t fock_assemble(const double* h, const double* J, const double* K, double* F, int64_t n, hipStream_t st);
hipError_t commutator(const double* M, double* e, int N, hipStream_t st);   // e = M - M^T
// Reductions over N x N matrices take a scratch `red` of red_elems(N) doubles.
int red_elems(int N);
hipError_t diis_dots(const double* const* es, int m, const double* enew, double* row, int64_t n, double* red,
                     hipStream_t st);
hipError_t diis_solve(const double* Bmat, int m, int ld, double* coef, hipStream_t st);
// DIIS inner products into the slot-indexed 8 x 8 matrix Bfull, and the m x m
// matrix of slots[0..m) gathered into Bm (ld 8); no host round trip.
hipError_t diis_prep(double* Bfull, const double* row, const int* slots, int m, int snew, double* Bm,
                     hipStream_t st);
hipError_t diis_combine(const double* const* Fs, const double* coef, int m, double* out, int64_t n, hipStream_t st);
hipError_t gershgorin(const double* F, int N, double* bounds, double* red, hipStream_t st);
hipError_t hash_matrix(double* R, int64_t n, uint32_t seed, hipStream_t st);
// ---- purification, one launch per step (tc2.hip).  part: 2 * tc2f_tiles(N)
// doubles per parity; state: 8 ints per parity ([0] countdown, [1] done,
// [2] steps run, [3] 1 if the latest X is in the step's output buffer).
// Step k reads parity k % 2 and writes parity (k + 1) % 2; out_id says which
// buffer the step writes (1: Y).
int tc2f_tiles(int N);
hipError_t tc2f_init(const double* F, const double* bounds, int N, double* X, double* part, int* state,
                     hipStream_t st);
hipError_t tc2f_step(const double* X, double* Y, int N, int n_occ, const double* part_in, double* part_out,
                     const int* st_in, int* st_out, int out_id, hipStream_t st);
hipError_t tc2f_final(double* X, const double* Y, int N, const int* state, hipStream_t st);
hipError_t energy_terms(const double* D, const double* h, const double* J, const double* K, int64_t n,
                        const double* enuc, double* out, double* red, hipStream_t st);
}  // namespace ri

namespace ri {
// ---- gradient (grad.hip).  Each contribution kernel runs on a fixed grid of
// GRAD_BLOCKS blocks and writes one partial gradient row [n_centres*3] per
// block into `part` (rows [row0, row0 + GRAD_BLOCKS)); grad_reduce sums rows.
constexpr int GRAD_BLOCKS = 1024;
hipError_t grad_one_electron(const ri_system* s, const double* D, const double* W, double* part, hipStream_t st);
hipError_t grad_metric(const ri_system* s, const double* Z, const double* c, double* part, hipStream_t st);
// Zx = -2 Xi Xi^T (lower 128-tiles) for Xi [n_aux][K], split over K through
// tmp (tmp_elems doubles of scratch).
hipError_t grad_metric_z(const double* Xi, int n_aux, int64_t K, double* tmp, int64_t tmp_elems, double* Zx,
                         hipStream_t st);
// Three-centre term.  (U^P C^T)_mu_nu (U^P = C Xi^P, [n_aux][N][n_occ]) is formed
// on MFMA for the lower 64 x 64 tiles, grad_slab(N, n_aux) auxiliary indices at
// a time, into WY (workspace of grad_slab * N * N doubles), and the derivative
// kernel reads it at the significant pairs.  For n_occ <= 128 the products run
// in a kernel that keeps C's tile rows in registers across 8 auxiliaries.
int grad_slab(int N, int n_aux);
// U[p] = C Xi^p for p < np: C [N][K], Xi [np][K][K] with symmetric blocks,
// U [np][N][K].
hipError_t u_products(const double* C, const double* Xi, int N, int K, int np, double* U, hipStream_t st);
hipError_t grad_three_centre(const ri_system* s, const int32_t* pairs, int64_t n_pairs, const double* U,
                             const double* C, int n_occ, const double* D, const double* c, double* WY,
                             double* part, hipStream_t st);
hipError_t grad_nuclear(const ri_system* s, double* part, hipStream_t st);
hipError_t grad_reduce(const double* part, int rows, int n_centres, double* grad, hipStream_t st);
hipError_t gamma_only(const double* Bc, const int32_t* pairs, int64_t n_pairs, int n_aux, int n_occ,
                      const double* C, double* dpair, double* gamma, hipStream_t st);
}  // namespace ri

namespace ri {
// ---- learned start (mlp.hip)
struct MlpWS { float *xh, *z1, *h1, *z2, *h2, *y, *dy, *part, *grad; __bf16* W2t; };
MlpWS carve_mlp(char* base, size_t cap, size_t& off, int64_t n);
hipError_t pair_features(const ri_system* s, const int32_t* pairs, int64_t n_pairs, float* feat, hipStream_t st);
hipError_t mlp_forward(const ri_mlp* net, const float* feat, int64_t n, float* y, int prec, const MlpWS& w,
                       hipStream_t st);
hipError_t mlp_train_step(const ri_mlp* net, float* m, float* v, int step, float lr, const float* feat,
                          const float* target, int64_t n, float* loss, const MlpWS& w, hipStream_t st);
hipError_t gather_density(int N, const int32_t* pairs, int64_t n_pairs, const double* D, float* d, hipStream_t st);
hipError_t scatter_density(int N, const int32_t* pairs, int64_t n_pairs, const float* d, double* D, hipStream_t st);
hipError_t pair_delta_features(const ri_system* s, const double* xyz_prev, const int32_t* pairs, int64_t n_pairs,
                               const double* D_prev, float* feat, hipStream_t st);
hipError_t density_change(int N, const int32_t* pairs, int64_t n_pairs, const double* Dn, const double* Dp,
                          float scale, float* d, hipStream_t st);
hipError_t density_add(int N, const int32_t* pairs, int64_t n_pairs, const float* d, double scale, const double* Dp,
                       double* Dout, hipStream_t st);
}  // namespace ri

namespace ri {
void set_hip_error(const char* text);   // text returned by ri_last_hip_error
// ---- batched SCF (many molecules per launch)
// Per-molecule state of a batched SCF, resident in device memory.  Batched
// kernels run over work items of all molecules: a per-kernel prefix table
// (device, n_mol + 1 ints) maps each linear block index to (molecule, local).
struct MolDesc {
    int N, n_aux, n_occ, nt, npad, ks, diis_n;
    int xs;       // X launch shape: 4 * (whole 16-row occupied tiles) + (trailing 4-row quads)
    int xs64;     // the FP64 X shape (final FP64 exchange after an FP32 SCF)
    int64_t n_pairs, ntl, rows_pad, chunk;
    double tol_E, tol_err;
    const int32_t* pairs;
    const double* Bc;
    const void* B;
    double *C, *J, *K, *gamma, *dpair, *part;
    void* Xt;
    double *S, *H, *LinvS, *F, *D, *T1, *T2, *E, *Fx, *X, *X2, *Y, *Cp, *Mo, *LinvM, *dinvM;
    double* Cq;   // C_occ zero-padded to [64 * nt][64], FP64 (or FP32 for FP32 exchange)
    double *dF[8], *dE[8];
    double *Bmat, *coef, *scal;
    int* state;   // 0 active, 1 iteration, 2 DIIS pushes, 3 converged, 4.. DIIS slot order [8], 14.. purification
};

// One member of a grouped FP64 GEMM: C = alpha op(A) op(B) + beta C.
struct GemmDesc {
    int M, N, K, tri;
    double alpha, beta;
    const double* A;
    const double* B;
    double* C;
    int64_t lda, ldb, ldc;
    const int* active;
    // sym: the product is symmetric (M == N): only the tiles on and above the
    // diagonal run, in row-major order, and every entry is also written to its
    // mirror position, so C comes out exactly symmetric
    int sym;
};
// tile: 64 (64 x 64 tiles) or 128 (128 x 128 tiles); prefix counts tiles of
// that size (t (t + 1) / 2 for a symmetric product).
hipError_t gemm_grouped(bool ta, bool tb, const GemmDesc* d, const int* prefix, int n, int total, hipStream_t s,
                        int tile = 64);

__device__ __forceinline__ void decode_item(const int* prefix, int n_mol, int L, int& mol, int& local) {
    int lo = 0, hi = n_mol;            // prefix[lo] <= L < prefix[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (prefix[mid] <= L) lo = mid; else hi = mid;
    }
    mol = lo;
    local = L - prefix[lo];
}

// batched Fock build pieces (fock.hip); `prec` is RI_FP64 or RI_FP32 for all molecules
// X for the molecules whose xs equals `xs` (one launch per shape present); prec may
// also be X_F64_B32 (FP64 shapes, Cq and Xt)
hipError_t x_transform_b(const MolDesc* d, const int* prefix, int n_mol, int total, int xs, int prec, hipStream_t st);
// Cq of every active molecule from its C (prefix counts 64-row blocks), in the
// exchange precision `prec`
hipError_t cpad_b(const MolDesc* d, const int* prefix, int n_mol, int total, int prec, hipStream_t st);
hipError_t syrk_b(const MolDesc* d, const int* prefix, int n_mol, int total, int prec, hipStream_t st);
hipError_t kreduce_b(const MolDesc* d, const int* prefix, int n_mol, int total, hipStream_t st);
hipError_t zero_tail_b(const MolDesc* d, const int* prefix, int n_mol, int total, int prec, hipStream_t st);
hipError_t gamma_j_b(const MolDesc* d, int n_mol, const int* pre_pairs, int tot_pairs, const int* pre_aux, int tot_aux,
                     const int* pre_n2, int tot_n2, hipStream_t st);
}  // namespace ri

namespace ri {
// ---- split-BF16 exchange (bf16.hip)
// compute units of the current device (256 if it cannot be queried); cached per device
int device_cus();
int bf16_parts(int prec);
int64_t bf16_R(int n_aux, int n_occ);
int64_t bf16_ct_elems(int N, int n_occ);
int64_t bf16_xb_elems(int N, int n_aux, int n_occ);
int bf16_split_count(int N, int n_aux, int n_occ);
hipError_t pack_b_bf16(const double* Bc, int64_t n_pairs, const int32_t* map, int N, int n_aux, void* B, int prec,
                       hipStream_t st);
hipError_t x_transform_bf16(const void* B, int prec, int N, int n_aux, int n_occ, const double* C, void* Ct,
                            void* Xb, hipStream_t st);
hipError_t k_syrk_bf16(const void* Xb, int prec, int N, int n_aux, int n_occ, double* part, int n_split, double* K,
                       hipStream_t st);
}  // namespace ri
