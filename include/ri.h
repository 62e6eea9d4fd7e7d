/*
 * ri.h - C ABI of libri, an MI355X (gfx950) implementation of the
 * resolution-of-the-identity Hartree-Fock hot path: RI J/K Fock builds and
 * the RI-HF analytic gradient (Stocks, Palethorpe, Barca, "Multi-GPU RI-HF
 * Energies and Analytic Gradients", arXiv 2407.19614).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Basis functions are normalised primitive s-Gaussians
 *   phi(r) = (2a/pi)^{3/4} exp(-a |r - A|^2); auxiliary functions likewise.
 *   One function per shell.
 * - All device pointers are allocated and owned by the caller; the library
 *   never allocates device memory.  Its only state is a cached compute-unit
 *   count per device, one side stream per device (made on first use, default
 *   priority) and the last HIP error text.  Scratch memory comes from `ws`
 *   (device, >= 256-byte aligned) of `ws_bytes` bytes, sized by
 *   ri_workspace_bytes().  Calls that take a `hipStream_t` enqueue their work
 *   on that stream (ri_fock_jk and ri_energy also fork part of it to the
 *   side stream and join it back into `stream`); only calls that return host
 *   scalars synchronise that stream.
 * - Matrices are row-major FP64 unless stated.  N = number of orbital basis
 *   functions, n_aux = number of auxiliary functions, n_occ = number of doubly
 *   occupied orbitals.
 * - Sign of exchange: K = +sum_P X^P X^P^T (positive semidefinite) with
 *   X^P = B^P C_occ; the Fock matrix is F = h + J - K.  The paper's exchange
 *   term (eq. k) is -K.
 * - Factor convention (eq. symmetric_ri / eq. biap): A = L L^T with L lower
 *   triangular, B^P = sum_Q [L^{-1}]_PQ (mu nu|Q).  The paper's A^L is L^{-T}.
 * - Errors: every entry point returns an ri_status; no exception crosses the
 *   ABI, nothing is printed and nothing aborts.  On RI_E_HIP the HIP error
 *   text is available from ri_last_hip_error().
 */
#ifndef RI_H
#define RI_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RI_OK = 0,
    RI_E_ARG = 1,          /* NULL pointer, negative or inconsistent size     */
    RI_E_NOT_PD = 2,       /* metric or overlap not positive definite         */
    RI_E_NO_CONV = 3,      /* SCF did not converge within max_iter            */
    RI_E_WORKSPACE = 4,    /* ws_bytes smaller than ri_workspace_bytes()      */
    RI_E_CAPACITY = 5,     /* pair capacity too small (count is returned)     */
    RI_E_HIP = 6,          /* a HIP runtime call failed                       */
    RI_E_UNSUPPORTED = 7,  /* option not supported (e.g. unknown precision)   */
    RI_E_NO_PURIFY = 8     /* purification of a Fock matrix did not reach an  */
                           /* idempotent projector within its step limit      */
} ri_status;

/* Storage precision of the packed B tensor and arithmetic of the X / K
 * contractions (project extension; FP64 is the paper's precision). */
typedef enum {
    RI_FP64 = 0,     /* B in FP64, FP64 MFMA                                  */
    RI_FP32 = 1,     /* B in FP32, FP32 MFMA, FP32 accumulation per P-chunk,  */
                     /* FP64 across chunks                                    */
    RI_BF16X3 = 2,   /* B split as hi + lo bfloat16; products hi*hi + hi*lo + */
                     /* lo*hi on BF16 MFMA with FP32 accumulation per chunk,  */
                     /* FP64 across chunks                                    */
    RI_BF16X6 = 3    /* three-part split hi + mid + lo; the six products whose */
                     /* part orders add to at most 2 (about FP32 accuracy)    */
} ri_precision;

/* Flag OR-ed into a precision argument (with RI_FP64 or RI_FP32 only): B is
 * not resident.  Every call that needs B decompresses the fitted tensor B_c
 * into packed tiles, RI_COMPRESSED_SLAB auxiliary functions at a time, in its
 * workspace (the per-iteration decompression of Algorithm 1), and B is passed
 * as NULL.  Results are identical to the resident form; workspace sizes from
 * ri_workspace_bytes with the same flag. */
#define RI_COMPRESSED 0x10
#define RI_COMPRESSED_SLAB 256

/* Flag OR-ed into the precision of ri_energy (with RI_FP32, RI_BF16X3 or
 * RI_BF16X6, resident B) and of the batched SCF calls (RI_FP32 only): the SCF
 * iterations run with the reduced-precision exchange; once converged, the
 * exchange matrix is rebuilt once in FP64 arithmetic at the converged density
 * (C, X and K in FP64; B is the FP32-stored B widened exactly on load, or,
 * for the split-BF16 forms, the FP64 fitted tensor B_c unpacked
 * RI_COMPRESSED_SLAB auxiliaries at a time), and the reported energy
 * (E_total, E_K) is the one with this K.  The energy is stationary in the
 * density, so the density's error from the reduced-precision iterations enters
 * it only to second order, while reduced-precision arithmetic in the exchange
 * shifts it to first order; what stays first order is the rounding of the B
 * the final build reads (FP32 for RI_FP32, none for the split-BF16 forms).
 * n_iter, converged, last_dE, max_err and the returned Fock matrix are those
 * of the reduced-precision iterations; a run that does not converge reports
 * their energies.  Workspaces hold FP64 Xt and C copies (sizes from the same
 * flag).  Other calls reject it (RI_E_UNSUPPORTED).
 * RI_BF16X3 SCF is offered only with this flag: two bfloat16 parts hold B
 * and C_occ to about 2^-17 relative, which alone moves the 8-centre
 * workload's energy by more than 1e-6 Eh. */
#define RI_FINAL_FP64 0x20

/* Molecular system.  The struct lives in host memory; every array is a
 * device pointer.  Positions in bohr. */
typedef struct {
    int32_t n_centres;
    int32_t n_fn;                 /* N                                       */
    int32_t n_aux;                /* N_aux                                   */
    int32_t n_occ;                /* doubly occupied orbitals                */
    const double* xyz;            /* [n_centres][3]                          */
    const double* Z;              /* [n_centres] nuclear charges             */
    const int32_t* fn_centre;     /* [N] centre index of each function       */
    const double* fn_exp;         /* [N] exponent of each function           */
    const int32_t* aux_centre;    /* [N_aux]                                 */
    const double* aux_exp;        /* [N_aux]                                 */
} ri_system;

/* Packed B tensor geometry.  B^P is symmetric in (mu, nu) (the paper's
 * Symmetry-utilisation section) and is stored as the lower triangle of
 * 64 x 64 tiles: tile (I, J), I >= J, has index I(I+1)/2 + J and holds
 * B^P[64I + r][64J + c] at offset r*64 + c; entries beyond N are zero.
 * Layout [n_aux][n_tiles][64*64] of the storage type (double or float).
 * The split-BF16 precisions store full square tiles instead (every I and
 * J), each as NS = 2 (BF16X3) or 3 (BF16X6) bfloat16 parts:
 * [n_aux][nt][nt][2][NS][64][32], part k of B^P[64I + r][64J + 32h + c] at
 * offset (h*NS + k)*2048 + r*32 + c of tile (I, J).
 * ri_packed_b_bytes() returns the size. */
#define RI_TILE 64
size_t ri_packed_b_bytes(int32_t N, int32_t n_aux, int32_t prec);

/* ri_build_3c - Schwarz screening of orbital pairs and the three-centre
 * integrals (mu nu|P) over the significant pairs.
 * Paper: definitions of the two- and three-centre ERIs (Notation section);
 * basis-function pair screening (Basis-function pair sparsity section): a
 * pair is dropped when (mu nu|mu nu) <= tau; Algorithm 1, three-centre ERI
 * computation for each auxiliary batch.
 *   pairs   [cap][2] int32 (device, out): significant pairs (mu, nu), mu >= nu,
 *           ordered by mu, then nu.
 *   cap     capacity of `pairs` (and the column count T was sized for).
 *   n_pairs (host, out): number of significant pairs.  If it exceeds cap the
 *           call returns RI_E_CAPACITY and writes nothing else.
 *   T       [n_aux][n_pairs] (device, out; row stride n_pairs), or NULL to
 *           only screen.
 * Synchronises `stream` once to read the pair count.
 * Workspace: ri_workspace_bytes(RI_OP_BUILD_3C, ...). */
int32_t ri_build_3c(const ri_system* sys, double tau, int32_t* pairs, int64_t cap,
                    int64_t* n_pairs, double* T, void* ws, size_t ws_bytes,
                    hipStream_t stream);

/* ri_metric_factor - the Coulomb metric A_PQ = (P|Q), its Cholesky factor
 * A = L L^T (FP64), the fitted tensor on compressed pairs
 * Bc = L^{-1} T (overwrites T in place), and the packed ("decompressed")
 * B tensor in precision `prec`.
 * Paper: eq. symmetric_ri and eq. biap (Cholesky of the metric, B formation);
 * Algorithm 1, the formation of B and its one-time decompression when memory
 * allows.
 *   T_inout [n_aux][n_pairs] in: (mu nu|P); out: Bc.
 *   L       [n_aux][n_aux] out: lower factor (upper triangle zeroed).
 *   Linv    [n_aux][n_aux] out: L^{-1} (lower).
 *   B       packed B (see above), out; may be NULL to skip packing (as for
 *           the compressed form, prec | RI_COMPRESSED).
 *   bad_pivot (host, out): -1, or the first auxiliary index whose pivot is
 *           not positive (then RI_E_NOT_PD is returned).
 * Synchronises `stream` once (pivot check). */
int32_t ri_metric_factor(const ri_system* sys, const int32_t* pairs, int64_t n_pairs,
                         double* T_inout, double* L, double* Linv, void* B, int32_t prec,
                         int64_t* bad_pivot, void* ws, size_t ws_bytes, hipStream_t stream);

/* ri_pack_b - the packed B tensor (layout above) in precision `prec` from
 * the fitted tensor on compressed pairs, as ri_metric_factor writes it: the
 * same B in a second precision without refactoring the metric.
 * Paper: Algorithm 1, the one-time decompression of B when memory allows.
 *   Bc      [n_aux][n_pairs] FP64 fitted tensor and pairs [n_pairs][2], as
 *           returned by ri_metric_factor / ri_build_3c (device, read).
 *   B       ri_packed_b_bytes(N, n_aux, prec) bytes (device, out; every byte
 *           is written).
 *   prec    RI_FP64, RI_FP32, RI_BF16X3 or RI_BF16X6, no flags
 *           (RI_E_UNSUPPORTED otherwise).
 * Workspace: ri_workspace_bytes(RI_OP_METRIC, N, n_aux, 0, n_pairs, prec).
 * Asynchronous: no host synchronisation. */
int32_t ri_pack_b(int32_t N, int32_t n_aux, const double* Bc, const int32_t* pairs, int64_t n_pairs,
                  void* B, int32_t prec, void* ws, size_t ws_bytes, hipStream_t stream);

/* ri_fock_jk - one RI Fock build: Coulomb J and exchange K for the density
 * D = 2 C_occ C_occ^T.
 * Paper: eq. j_ri (gamma_P = sum B^P_mu_nu D_mu_nu, J = sum_P gamma_P B^P),
 * eq. k_ri_2 and eq. tp (X^P = B^P C_occ, K = sum_P X^P X^P^T), Algorithm 1
 * Fock-build loop, symmetric GEMM for the lower triangle of K (Symmetry
 * utilisation section).
 *   B       packed B in precision `prec` (from ri_metric_factor), or NULL
 *           with prec | RI_COMPRESSED: X^P is then formed slab by slab from
 *           Bc (Algorithm 1's per-iteration decompression).
 *   Bc      [n_aux][n_pairs] FP64 fitted tensor on compressed pairs, and
 *   pairs   [n_pairs][2]: gamma and J are formed from these in FP64 for
 *           every precision.
 *   C_occ   [N][n_occ] row-major.
 *   J, K    [N][N] out, full symmetric.
 *   gamma   [n_aux] out (may be NULL).
 * Asynchronous: no host synchronisation.  The gamma/J part runs on a
 * library-owned side stream of the current device (one per device, default
 * priority, created on first use), concurrently with the exchange (for the
 * split-BF16 forms with the SYRK only, after X); `stream` waits for it
 * before any later work on `stream`, so the outputs are ordered on `stream`
 * as if all work ran there.  Also used by ri_energy's SCF loop. */
int32_t ri_fock_jk(int32_t N, int32_t n_aux, int32_t n_occ, const void* B, int32_t prec,
                   const double* Bc, const int32_t* pairs, int64_t n_pairs,
                   const double* C_occ, double* J, double* K, double* gamma,
                   void* ws, size_t ws_bytes, hipStream_t stream);

/* ri_fock_jk_noalloc - ri_fock_jk for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments without the workspace, same kernels and
 * results (bit for bit).  Scratch is a static device array of
 * RI_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on
 * until the process ends; the call returns RI_E_WORKSPACE when the build
 * needs more (ri_workspace_bytes(RI_OP_FOCK, ...) above that size: N = 200
 * with N_aux = 600 and n_occ = 20 fits in FP64, N = 240 with 720 and 24 does
 * not).  It makes no allocation of any kind: the whole build runs on
 * `stream` (no side stream, no events).  The first call on a device looks up
 * the array's device address once.  Every call on a device shares that
 * device's array and leaves its contents behind; nothing in it needs to start
 * at zero (each call writes every scratch element it reads).  Calls that
 * overlap in time on one device (other streams or threads) race on the array
 * and must be serialised by the caller.  Asynchronous. */
#define RI_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int32_t ri_fock_jk_noalloc(int32_t N, int32_t n_aux, int32_t n_occ, const void* B, int32_t prec,
                           const double* Bc, const int32_t* pairs, int64_t n_pairs,
                           const double* C_occ, double* J, double* K, double* gamma, hipStream_t stream);

/* ri_fock_jk_timed - ri_fock_jk with phase events, for measurement.
 * Same computation, arguments and schedule as ri_fock_jk (paper: eq. j_ri,
 * eq. k_ri_2, eq. tp, Algorithm 1 Fock-build loop): the gamma/J contraction
 * runs on the library's side stream beside the exchange.  Records
 *   events[0] on `stream` before both parts;
 *   events[1] on the side stream after gamma/J (gamma/J = events[0..1];
 *             for the split-BF16 forms the side stream forks after X, and
 *             gamma/J = events[2..1], beside the SYRK);
 *   events[2] on `stream` after the exchange half-transform X^P = B^P C_occ
 *             (X = events[0..2], measured while gamma/J runs beside it);
 *   events[3] on `stream` after the K = sum X X^T SYRK, its reduction and
 *             the wait for gamma/J (SYRK = events[2..3]).
 * events: four events created by the caller (host array).  RI_E_HIP if the
 * side stream is not available. */
int32_t ri_fock_jk_timed(int32_t N, int32_t n_aux, int32_t n_occ, const void* B, int32_t prec,
                         const double* Bc, const int32_t* pairs, int64_t n_pairs,
                         const double* C_occ, double* J, double* K, double* gamma,
                         void* ws, size_t ws_bytes, hipStream_t stream, hipEvent_t* events);

typedef struct {
    int32_t max_iter;      /* default 100                                       */
    int32_t diis_n;        /* DIIS subspace size, 1..8 (default 6)              */
    double tol_E;          /* |E_k - E_{k-1}| threshold (default 1e-10)         */
    double tol_err;        /* max |F D S - S D F| threshold (default 1e-8)      */
    int32_t guess_kind;    /* 0 core Hamiltonian; 1 C_occ [N][n_occ] in `guess`;*/
                           /* 2 density D [N][N] in `guess`: start from the    */
                           /*   n_occ largest solutions of (S D S) v = l S v;  */
                           /* 3 density D [N][N] in `guess`: start from the    */
                           /*   occupied space of F(D) = h + J(D) - K(D), the  */
                           /*   Fock matrix of the density itself             */
    int32_t max_purify;    /* step limit of each trace-correcting purification */
                           /* (0: the default, 200 for ri_energy; for         */
                           /* ri_energy_batched, whose launch sequence is     */
                           /* fixed, 128 at the core-Hamiltonian start and in */
                           /* each iteration);                                */
                           /* a purification whose |tr X - tr X^2| has not    */
                           /* fallen below 1e-11 n_occ by then fails          */
} ri_scf_opts;

typedef struct {
    double E_total, E_nuc, E_1e, E_J, E_K;
    int32_t n_iter, converged;
    double last_dE, max_err;
} ri_scf_result;

/* ri_fock_jk_density - Coulomb J and exchange K of a density matrix D
 * given without orbitals (a density start such as a superposition of atomic
 * densities, or a predicted density).
 * Paper: eq. j_ri for J (gamma_P = sum B^P_mu_nu D_mu_nu); exchange in its
 * density form, eq. k with the RI factorisation eq. ri_eri, which reads
 * K = 1/2 sum_P B^P D B^P (the C_occ-factored eq. tp / eq. k_ri_2 needs
 * orbitals; the Exchange-build remark notes that a density start makes the
 * first build slower).  Cost 4 N^3 N_aux FP64 MFMA flops, against
 * 3 N^2 n_occ N_aux for ri_fock_jk.
 *   Bc, pairs  as from ri_metric_factor (B itself is not used).
 *   D          [N][N] device FP64, symmetric (its symmetric part is used).
 *   J, K       [N][N] out; gamma [n_aux] out or NULL.
 * Workspace: ri_workspace_bytes(RI_OP_FOCK_DENSITY, N, n_aux, 1, n_pairs, RI_FP64).
 * Asynchronous. */
int32_t ri_fock_jk_density(int32_t N, int32_t n_aux, const double* Bc, const int32_t* pairs, int64_t n_pairs,
                           const double* D, double* J, double* K, double* gamma,
                           void* ws, size_t ws_bytes, hipStream_t stream);

/* ri_energy - closed-shell RI-HF SCF.
 * Paper: Roothaan equations (Energy formulation section), Fock build
 * (eq. fock_build with the RI J/K of ri_fock_jk), DIIS and a new set of
 * occupied orbitals each iteration (Algorithm 1, SCF loop).
 * The occupied space of each extrapolated Fock matrix (the n_occ lowest
 * orbitals of F C = S C eps) is obtained as the spectral projector by
 * trace-correcting purification, all on the GPU.
 *   B, prec   as for ri_fock_jk (B may be NULL with prec | RI_COMPRESSED);
 *             prec may also be RI_FP32, RI_BF16X3 or RI_BF16X6 with
 *             RI_FINAL_FP64; RI_BF16X3 without it is rejected
 *             (RI_E_UNSUPPORTED, see RI_FINAL_FP64).
 *   guess     device C_occ [N][n_occ] (guess_kind 1) or D [N][N] (guess_kind 2),
 *             else NULL.
 *   C_occ     [N][n_occ] out: orthonormal (C^T S C = 1) occupied orbitals
 *             spanning the converged occupied space (not canonical).
 *   F_out     [N][N] out: Fock matrix built from C_occ.
 *   D_out     [N][N] out (may be NULL): D = 2 C_occ C_occ^T.
 *   res       (host, out).
 * Returns RI_E_NO_CONV (with `res` filled) when max_iter is reached, and
 * RI_E_NO_PURIFY (with `res` filled up to the last completed iteration,
 * converged = 0) when a purification fails (see max_purify), e.g. for a Fock
 * matrix with no gap between its n_occ-th and next eigenvalue.
 * Synchronises the stream once per iteration. */
int32_t ri_energy(const ri_system* sys, const void* B, int32_t prec, const double* Bc,
                  const int32_t* pairs, int64_t n_pairs, const ri_scf_opts* opts,
                  const double* guess, double* C_occ, double* F_out, double* D_out,
                  ri_scf_result* res, void* ws, size_t ws_bytes, hipStream_t stream);

/* ri_gradient - analytic RI-HF nuclear gradient at a converged SCF.
 * Paper: eq. hf_gradient and eq. rihf_gradient with the Coulomb (L^P) and
 * exchange (X_ij^P) coefficients of the Gradient-formulation section,
 * Algorithm 2.  With D = 2 C C^T:
 *   c = L^{-T} gamma, Xi^P_ij = [L^{-T} B_ij]_P, B^P_ij = (C^T B^P C)_ij,
 *   Y^P = c_P D - 2 C Xi^P C^T,  Z = c c^T - 2 sum_ij Xi_ij Xi_ij^T,
 *   W = (1/2) D F D (= 2 C eps C^T at convergence),
 *   g = sum D h' - sum W S' + sum Y (mu nu|P)' - 1/2 sum Z (P|Q)' + E_nn'.
 *   B, prec, Bc, pairs, Linv as returned by ri_metric_factor (B may be NULL
 *            with prec | RI_COMPRESSED).  With RI_FP64 or RI_FP32 the
 *            half-transform X^P = B^P C for B_ij reads B in that precision.
 *            With RI_BF16X3 or RI_BF16X6, B is not read (it may be NULL):
 *            B_ij, Xi and every sum are formed in FP64 from Bc, unpacked
 *            RI_COMPRESSED_SLAB auxiliaries at a time as for RI_COMPRESSED,
 *            since B_ij and Xi enter the gradient linearly and the split
 *            parts carry B only to 2^-17 (or 2^-25); the result is the FP64
 *            gradient at the orbitals the split-BF16 SCF converged to.
 *   C_occ, F  converged orbitals and Fock matrix from ri_energy.
 *   grad     [n_centres][3] out, Eh/bohr, including nuclear repulsion.
 * Asynchronous. */
int32_t ri_gradient(const ri_system* sys, const int32_t* pairs, int64_t n_pairs,
                    const void* B, int32_t prec, const double* Bc, const double* Linv,
                    const double* C_occ, const double* F, double* grad,
                    void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned SCF start (project extension, not proposed by the paper; the
 * paper starts each molecular-dynamics SCF from the previous step's orbitals,
 * AIMD section).  A 3-layer MLP maps per-pair features to density-matrix
 * elements D_mu_nu; ri_energy then starts from the occupied space of that
 * density (guess_kind 2).
 * Pair features (RI_MLP_NFEAT = 8) of (mu, nu) with centres A, B, exponents a, b:
 *   |A-B|, ln max(a,b), ln min(a,b), [A == B], exp(-(ab/(a+b))|A-B|^2),
 *   max and min over {A, B} of c_X = sum_{C != X} exp(-|R_X - R_C|^2 / 8),
 *   sum_C exp(-|P - R_C|^2 / 4) with P = (aA + bB)/(a + b).
 * Network: x = (f - mu)/sigma; h1 = silu(x W1 + b1); h2 = silu(h1 W2 + b2);
 *   y = h2 w3 + b3; silu(z) = z/(1+exp(-z)).  Parameters are one flat FP32
 *   device array laid out as W1 [8][256], b1 [256], W2 [256][256], b2 [256],
 *   w3 [256], b3 [1] (offsets RI_MLP_OFF_*). */
#define RI_MLP_NFEAT 8
#define RI_MLP_WIDTH 256
#define RI_MLP_OFF_W1 0
#define RI_MLP_OFF_B1 (RI_MLP_OFF_W1 + RI_MLP_NFEAT * RI_MLP_WIDTH)
#define RI_MLP_OFF_W2 (RI_MLP_OFF_B1 + RI_MLP_WIDTH)
#define RI_MLP_OFF_B2 (RI_MLP_OFF_W2 + RI_MLP_WIDTH * RI_MLP_WIDTH)
#define RI_MLP_OFF_W3 (RI_MLP_OFF_B2 + RI_MLP_WIDTH)
#define RI_MLP_OFF_B3 (RI_MLP_OFF_W3 + RI_MLP_WIDTH)
#define RI_MLP_NPARAM (RI_MLP_OFF_B3 + 1)
enum { RI_MLP_FP32 = 0, RI_MLP_BF16 = 1 };

typedef struct {
    float* params;          /* device [RI_MLP_NPARAM]                          */
    const float* mu;        /* device [RI_MLP_NFEAT] feature shift             */
    const float* sigma;     /* device [RI_MLP_NFEAT] feature scale             */
} ri_mlp;

/* ri_pair_features - features of each listed pair.
 *   feat [n_pairs][RI_MLP_NFEAT] FP32 (device, out).  Asynchronous. */
int32_t ri_pair_features(const ri_system* sys, const int32_t* pairs, int64_t n_pairs, float* feat,
                         hipStream_t stream);

/* ri_mlp_forward - y[n] = MLP(feat[n]).  prec RI_MLP_FP32, or RI_MLP_BF16
 * (the 256 x 256 layer with BF16 operands and FP32 accumulation).
 * Workspace: ri_workspace_bytes(RI_OP_MLP, .., n_pairs = n, ..). */
int32_t ri_mlp_forward(const ri_mlp* net, const float* feat, int64_t n, float* y, int32_t prec,
                       void* ws, size_t ws_bytes, hipStream_t stream);

/* ri_mlp_train_step - one Adam step (beta 0.9 / 0.999, eps 1e-8, step >= 1)
 * on the mean squared error of the FP32 forward against target[n].
 *   adam_m, adam_v [RI_MLP_NPARAM] device moments (zero before step 1).
 *   loss   device float (out): the loss before the update.
 *   grad   device [RI_MLP_NPARAM] (out, may be NULL): the loss gradient. */
int32_t ri_mlp_train_step(const ri_mlp* net, float* adam_m, float* adam_v, int32_t step, float lr,
                          const float* feat, const float* target, int64_t n, float* loss, float* grad,
                          void* ws, size_t ws_bytes, hipStream_t stream);

/* ri_density_from_pairs - dense symmetric D [N][N] (device, out, FP64) with
 * D_mu_nu = D_nu_mu = d[q] for pair q = (mu, nu) and zero elsewhere. */
int32_t ri_density_from_pairs(int32_t N, const int32_t* pairs, int64_t n_pairs, const float* d,
                              double* D, hipStream_t stream);

/* ri_density_to_pairs - d[q] = (float) D[mu][nu] for each listed pair q. */
int32_t ri_density_to_pairs(int32_t N, const int32_t* pairs, int64_t n_pairs, const double* D, float* d,
                            hipStream_t stream);

/* Start along a geometry sequence from the previous geometry's converged
 * density D' plus a predicted change (the network trained on the change
 * between consecutive geometries of the sequence).
 * Paper: the molecular-dynamics start from the previous step's solution
 * (Ab Initio Molecular Dynamics subsection of the algorithm section); the predicted
 * change on top of it is this library's extension.  Each of the three calls
 * returns RI_E_ARG for invalid sizes or NULL buffers and RI_E_HIP when its
 * launch fails; all pointers are device memory owned by the caller.
 * ri_pair_delta_features - features of each listed pair for that change,
 * between the previous positions xyz_prev (device [n_centres][3]; the basis
 * is sys's) and sys->xyz, with f4, c_X and f7 as for ri_pair_features:
 *   g0 = D'[mu][nu], g1 = change of |A - B|, g2 = change of f4,
 *   g3 = ln max(a,b), g4 = ln min(a,b), g5 = [A == B],
 *   g6 = change of c_A + c_B, g7 = change of f7.
 *   D_prev [N][N] device FP64; feat [n_pairs][RI_MLP_NFEAT] FP32 (out). */
int32_t ri_pair_delta_features(const ri_system* sys, const double* xyz_prev, const int32_t* pairs, int64_t n_pairs,
                               const double* D_prev, float* feat, hipStream_t stream);

/* ri_density_change_pairs - d[q] = scale (D_new - D_prev)[mu][nu] for each
 * listed pair q (training targets of the change). */
int32_t ri_density_change_pairs(int32_t N, const int32_t* pairs, int64_t n_pairs, const double* D_new,
                                const double* D_prev, float scale, float* d, hipStream_t stream);

/* ri_density_add_pairs - D_out = D_prev, except D_out[mu][nu] = D_out[nu][mu]
 * = D_prev[mu][nu] + scale d[q] on each listed pair q (the start density).
 * D_out must not alias D_prev. */
int32_t ri_density_add_pairs(int32_t N, const int32_t* pairs, int64_t n_pairs, const float* d, double scale,
                             const double* D_prev, double* D_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched SCF (project extension): many independent molecules advance through
 * the SCF of ri_energy in lockstep, each step one launch over all molecules,
 * optionally replayed from a captured HIP graph.  Per molecule the caller
 * supplies the outputs of ri_build_3c / ri_metric_factor. */
typedef struct {
    const void* B;          /* packed B in the batch precision                 */
    const double* Bc;       /* [n_aux][n_pairs] FP64 fitted tensor              */
    const int32_t* pairs;   /* [n_pairs][2]                                     */
    int64_t n_pairs;
    double* C_occ;          /* [N][n_occ] out                                   */
    double* F;              /* [N][N] out, or NULL                              */
} ri_batch_mol;


/* Workspace bytes for ri_energy_batched (0 on invalid input).  Supported:
 * prec RI_FP64, RI_FP32 or RI_FP32 | RI_FINAL_FP64, n_occ <= 64 for every
 * molecule. */
size_t ri_energy_batched_workspace(int32_t n_mol, const ri_system* sys, const ri_batch_mol* mol, int32_t prec);

/* Launch shapes of the batched SCF per size bucket.  Molecule m belongs to
 * bucket b = ceil(N_m / 128) - 1, clamped to n_buckets - 1.
 *   gemm_tile[b]   64 or 128: tile edge of the grouped FP64 GEMMs whose three
 *                  dimensions are N (orthogonalisation, purification squares,
 *                  F D and F D S products).
 *   syrk_split[b]  1 .. RI_TUNE_MAX_SPLIT: pieces the exchange SYRK reduction index
 *                  (n_aux * n_occ) is split into.
 *   gemm_ms[b], syrk_ms[b]  (filled by ri_batch_autotune) the measured time
 *                  of the chosen shape on the bucket's molecules, in ms.
 * Host memory, owned by the caller. */
#define RI_TUNE_BUCKETS 8
#define RI_TUNE_MAX_SPLIT 16
typedef struct {
    int32_t n_buckets;
    int32_t gemm_tile[RI_TUNE_BUCKETS];
    int32_t syrk_split[RI_TUNE_BUCKETS];
    float gemm_ms[RI_TUNE_BUCKETS];
    float syrk_ms[RI_TUNE_BUCKETS];
} ri_batch_tuning;

/* ri_batch_autotune - choose ri_batch_tuning for a batch by timing each
 * candidate shape (GEMM tile 64 / 128 on the purification square X X; SYRK
 * split 16, 8, 4, 2, 1 including its reduction, stopping at the first candidate
 * 1.1x slower than the best) with HIP events on the batch's own molecules of
 * each bucket, and keeping the fastest.  Takes the same
 * arguments and workspace as ri_energy_batched (sized by
 * ri_energy_batched_workspace) and leaves no result in it; C_occ and F of
 * mol are not touched.  Buckets with no molecule get the defaults (tile 64,
 * split from the reduction length).  Synchronises the stream. */
int32_t ri_batch_autotune(int32_t n_mol, const ri_system* sys, const ri_batch_mol* mol, int32_t prec,
                          ri_batch_tuning* out, void* ws, size_t ws_bytes, hipStream_t stream);

/* ri_energy_batched - closed-shell RI-HF SCF (as ri_energy, core-Hamiltonian
 * start) for n_mol molecules at once.
 * Paper: Roothaan equations and Algorithm 1 SCF loop, applied per molecule.
 *   sys, mol   host arrays [n_mol] (the pointers inside are device pointers).
 *   use_graph  1: capture one iteration as a HIP graph and replay it.
 *   tuning     launch shapes per size bucket (from ri_batch_autotune), or
 *              NULL for the defaults; RI_E_ARG if a value is out of range.
 *   prec       RI_FP64, RI_FP32, or RI_FP32 | RI_FINAL_FP64.
 *   res        host [n_mol] (out).
 * A molecule whose purification fails (opts->max_purify) stops iterating and
 * reports converged = 0.  Returns RI_E_NO_PURIFY if that happened to any
 * molecule, else RI_E_NO_CONV if any molecule did not converge (all results
 * filled).
 * Synchronises the stream once per iteration. */
int32_t ri_energy_batched(int32_t n_mol, const ri_system* sys, const ri_batch_mol* mol, int32_t prec,
                          const ri_scf_opts* opts, int32_t use_graph, const ri_batch_tuning* tuning,
                          ri_scf_result* res, void* ws, size_t ws_bytes, hipStream_t stream);

/* ri_md_verlet - one half of a velocity-Verlet step of the nuclei
 * (Born-Oppenheimer dynamics in the NVE ensemble; paper: Ab Initio Molecular
 * Dynamics subsection).  With a = -grad / mass (atomic units: bohr, electron
 * masses, Eh/bohr; dt in atomic time units):
 *   stage 0: vel += (dt/2) a, then xyz += dt vel   (before the new forces)
 *   stage 1: vel += (dt/2) a                       (with the new forces)
 *   mass [n_atoms], grad/xyz/vel [n_atoms][3]: device FP64.  xyz and vel are
 *   updated in place.  RI_E_ARG if dt <= 0 or stage is not 0 or 1. */
int32_t ri_md_verlet(int32_t n_atoms, double dt, const double* mass, const double* grad, double* xyz,
                     double* vel, int32_t stage, hipStream_t stream);

/* ri_md_kinetic - *ekin (device FP64, out) = sum_a 1/2 mass_a |vel_a|^2,
 * summed in a fixed order. */
int32_t ri_md_kinetic(int32_t n_atoms, const double* mass, const double* vel, double* ekin, hipStream_t stream);

/* Operation codes for ri_workspace_bytes.  For RI_OP_MLP, n_pairs is the
 * number of feature rows per call. */
enum { RI_OP_BUILD_3C = 0, RI_OP_METRIC = 1, RI_OP_FOCK = 2, RI_OP_ENERGY = 3,
       RI_OP_GRADIENT = 4, RI_OP_MLP = 5, RI_OP_FOCK_DENSITY = 6 };

/* Bytes of workspace an operation needs (0 on invalid arguments). */
size_t ri_workspace_bytes(int32_t op, int32_t N, int32_t n_aux, int32_t n_occ,
                          int64_t n_pairs, int32_t prec);

/* Human-readable text for a status code. */
const char* ri_status_str(int32_t status);

/* Text of the last HIP error seen by this thread ("" if none). */
const char* ri_last_hip_error(void);

/* Library version string. */
const char* ri_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RI_H */
