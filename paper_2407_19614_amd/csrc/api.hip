// C-ABI entry points of libri: argument checks, workspace carving and the
// sequencing of kernels on the caller's stream.
#include "kernels.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace {

thread_local std::string g_hip_err;

int32_t hip_status(hipError_t e) {
    if (e == hipSuccess) return RI_OK;
    g_hip_err = hipGetErrorString(e);
    return RI_E_HIP;
}

#define HIPC(x)                                          \
    do {                                                 \
        hipError_t _e = (x);                             \
        if (_e != hipSuccess) return hip_status(_e);     \
    } while (0)

// Bump allocator over the caller's workspace.  In dry mode it only counts
// bytes, so ri_workspace_bytes() and the entry points share one layout.
struct Arena {
    char* base;
    size_t cap;
    size_t off = 0;
    bool dry;
    template <class T>
    T* take(int64_t n) {
        size_t b = ((size_t)(n < 0 ? 0 : n) * sizeof(T) + 255) & ~(size_t)255;
        size_t o = off;
        off += b;
        return dry ? nullptr : (T*)(base + o);
    }
    // the size ri_workspace_bytes reports is off + 256
    bool ok() const { return dry || off + 256 <= cap; }
};

bool valid_sys(const ri_system* s) {
    return s && s->n_centres > 0 && s->n_fn > 0 && s->n_aux > 0 && s->n_occ > 0 && s->n_occ <= s->n_fn &&
           s->xyz && s->Z && s->fn_centre && s->fn_exp && s->aux_centre && s->aux_exp;
}

size_t elem_size(int prec) { return prec == RI_FP64 ? 8 : (prec == RI_FP32 ? 4 : 2); }
bool is_bf16(int prec) { return prec == RI_BF16X3 || prec == RI_BF16X6; }

// A precision argument: an ri_precision, optionally with RI_COMPRESSED (FP64 / FP32 only).
struct Prec {
    int base;
    bool comp, fin, ok;
};
// fin (RI_FINAL_FP64) is accepted where allow_fin is set, with resident FP32
// or split-BF16 B only
Prec split_prec(int32_t p, bool allow_fin = false) {
    Prec r{p & ~(RI_COMPRESSED | RI_FINAL_FP64), (p & RI_COMPRESSED) != 0, (p & RI_FINAL_FP64) != 0, true};
    if (r.base < 0 || r.base > 3) r.ok = false;
    if (r.comp && r.base != RI_FP64 && r.base != RI_FP32) r.ok = false;
    if (r.fin && (!allow_fin || r.base == RI_FP64 || r.comp)) r.ok = false;
    return r;
}
int comp_slab(int n_aux) { return std::min(RI_COMPRESSED_SLAB, (n_aux + 1) / 2 * 2); }

// ---------------------------------------------------------------- layouts
struct BuildWS { int32_t* counts; int64_t* offsets; };
BuildWS carve_build(Arena& a, int N) { return {a.take<int32_t>(N), a.take<int64_t>(N + 1)}; }

constexpr int64_t BC_CHUNK = 8192;
struct MetricWS { double* dinv; double* band; int* bad; int32_t* map; double* tmp; };
MetricWS carve_metric(Arena& a, int N, int n_aux, int64_t n_pairs) {
    MetricWS w;
    w.dinv = a.take<double>((int64_t)((n_aux + 63) / 64) * 4096);
    w.band = a.take<double>((int64_t)((n_aux + 63) / 64) * 4 * 4096);
    w.bad = a.take<int>(1);
    w.map = a.take<int32_t>((int64_t)N * N);
    w.tmp = nullptr;
    return w;
}

// Slab buffers of the compressed form: pair map and one slab of packed tiles.
struct SlabWS {
    int32_t* map = nullptr;
    void* Bs = nullptr;
    int slab = 0;
};
SlabWS carve_slab(Arena& a, int N, int n_aux, int prec, bool comp) {
    SlabWS w;
    if (!comp) return w;
    w.slab = comp_slab(n_aux);
    w.map = a.take<int32_t>((int64_t)N * N);
    w.Bs = a.take<char>((int64_t)w.slab * ri::tile_elems(N) * (int64_t)elem_size(prec));
    return w;
}

// X^T = (B^P C)^T for all P; from resident packed B, or (B == nullptr) slab by
// slab from B_c: unpack RI_COMPRESSED_SLAB auxiliaries into packed tiles, then
// transform them into their rows of X^T.
hipError_t x_any(const void* B, int prec, int N, int n_aux, int n_occ, const double* C, double* Cp, void* Xt,
                 const double* Bc, const int32_t* pairs, int64_t n_pairs, const SlabWS& sw, hipStream_t st) {
    if (B) return ri::x_transform(B, prec, N, n_aux, n_occ, C, Cp, Xt, st);
    if (!sw.Bs) return hipErrorInvalidValue;
    RI_TRY(ri::pair_map(pairs, n_pairs, N, sw.map, st));
    const int64_t row_bytes = (int64_t)ri::xt_ld(N) * (int64_t)elem_size(prec);
    for (int P0 = 0; P0 < n_aux; P0 += sw.slab) {
        const int ns = std::min(sw.slab, n_aux - P0);
        RI_TRY(ri::pack_b(Bc + (int64_t)P0 * n_pairs, n_pairs, sw.map, N, ns, sw.Bs, prec, st));
        RI_TRY(ri::x_transform(sw.Bs, prec, N, ns, n_occ, C, Cp, (char*)Xt + (int64_t)P0 * n_occ * row_bytes, st));
    }
    return hipSuccess;
}

struct FockWS { void* Xt; double* part; double* dpair; double* jpart; double* gamma; double* Cp; int ks, js; SlabWS sw; };
FockWS carve_fock(Arena& a, int N, int n_aux, int n_occ, int64_t n_pairs, int prec, bool comp = false) {
    FockWS w;
    w.sw = carve_slab(a, N, n_aux, prec, comp);
    const int Npad = ri::xt_ld(N);
    w.js = ri::j_split_count(n_aux);
    if (is_bf16(prec)) {
        const int ns = ri::bf16_parts(prec);
        w.ks = ri::bf16_split_count(N, n_aux, n_occ);
        w.Xt = a.take<char>(ri::bf16_xb_elems(N, n_aux, n_occ) * ns * 2);
        w.part = a.take<double>((int64_t)w.ks * Npad * Npad);
        w.dpair = a.take<double>(std::max<int64_t>(n_pairs, 1));
        w.jpart = a.take<double>((int64_t)w.js * std::max<int64_t>(n_pairs, 1));
        w.gamma = a.take<double>(n_aux);
        w.Cp = a.take<double>(ri::bf16_ct_elems(N, n_occ) * ns / 4 + 1);   // bf16 parts of C^T
        return w;
    }
    w.ks = ri::k_split_count(N, n_aux, n_occ);
    w.Xt = a.take<char>(ri::xt_rows(n_aux, n_occ) * Npad * (int64_t)(prec == RI_FP64 ? 8 : 4));
    w.part = a.take<double>((int64_t)w.ks * Npad * Npad);
    w.dpair = a.take<double>(std::max<int64_t>(n_pairs, 1));
    w.jpart = a.take<double>((int64_t)w.js * std::max<int64_t>(n_pairs, 1));
    w.gamma = a.take<double>(n_aux);
    w.Cp = a.take<double>(ri::cpad_elems(N, n_occ));
    return w;
}

// Fock build from a density matrix (no orbitals): pair weights, gamma/J
// buffers, and the slab buffers of K = 1/2 sum_P B^P D B^P.
constexpr int DENSITY_SLAB = 8;
struct DensityWS {
    double *dpair, *jpart, *gamma, *Bf, *Y;
    int32_t* map;
    int js, slab;
};
DensityWS carve_density(Arena& a, int N, int n_aux, int64_t n_pairs) {
    DensityWS w;
    const int64_t n2 = (int64_t)N * N;
    w.js = ri::j_split_count(n_aux);
    w.slab = std::min(DENSITY_SLAB, n_aux);
    w.dpair = a.take<double>(std::max<int64_t>(n_pairs, 1));
    w.jpart = a.take<double>((int64_t)w.js * std::max<int64_t>(n_pairs, 1));
    w.gamma = a.take<double>(n_aux);
    w.map = a.take<int32_t>(n2);
    w.Bf = a.take<double>(w.slab * n2);
    w.Y = a.take<double>(w.slab * n2);
    return w;
}

hipError_t jk_density(const double* Bc, const int32_t* pairs, int64_t n_pairs, int N, int n_aux, const double* D,
                      double* J, double* K, double* gamma, const DensityWS& w, hipStream_t st) {
    RI_TRY(ri::dpair_density(pairs, n_pairs, D, N, w.dpair, st));
    RI_TRY(ri::gamma_j_pairs(Bc, pairs, n_pairs, N, n_aux, w.dpair, gamma ? gamma : w.gamma, w.jpart, w.js, J, st));
    return ri::k_density(Bc, pairs, n_pairs, N, n_aux, D, w.map, w.Bf, w.Y, w.slab, K, st);
}

struct EnergyWS {
    double *S, *H, *Ls, *LinvS, *J, *K, *F, *D, *T1, *T2, *E, *Fx, *X, *X2;
    double *dF[8], *dE[8];
    double *Bmat, *Bfull, *coef, *row, *Y, *Cp, *R, *Mo, *LinvM, *dinvS, *dinvM, *scal, *red, *tpart;
    int *bad, *tst;
    FockWS fock;
    FockWS fin;   // final FP64 exchange build of the split-BF16 forms: FP64 Xt and slabs of B_c
    DensityWS dens;
};
EnergyWS carve_energy(Arena& a, int N, int n_aux, int n_occ, int64_t n_pairs, int prec, int diis_n,
                      bool comp = false, bool fin_slab = false) {
    EnergyWS w;
    const int64_t n2 = (int64_t)N * N;
    double** mats[] = {&w.S, &w.H, &w.Ls, &w.LinvS, &w.J, &w.K, &w.F, &w.D, &w.T1, &w.T2, &w.E, &w.Fx, &w.X, &w.X2};
    for (double** m : mats) *m = a.take<double>(n2);
    for (int i = 0; i < 8; ++i) {
        w.dF[i] = i < diis_n ? a.take<double>(n2) : nullptr;
        w.dE[i] = i < diis_n ? a.take<double>(n2) : nullptr;
    }
    w.Bmat = a.take<double>(64);
    w.Bfull = a.take<double>(64);
    w.coef = a.take<double>(8);
    w.row = a.take<double>(8);
    w.Y = a.take<double>((int64_t)N * n_occ);
    w.Cp = a.take<double>((int64_t)N * n_occ);
    w.R = a.take<double>((int64_t)N * n_occ);
    w.Mo = a.take<double>((int64_t)n_occ * n_occ);
    w.LinvM = a.take<double>((int64_t)n_occ * n_occ);
    w.dinvS = a.take<double>((int64_t)((N + 63) / 64) * 4096);
    w.dinvM = a.take<double>((int64_t)((n_occ + 63) / 64) * 4096);
    w.scal = a.take<double>(32);
    w.red = a.take<double>(ri::red_elems(N));   // reduction partials
    w.tpart = a.take<double>(4 * (int64_t)ri::tc2f_tiles(N));   // purification partial sums, two parities
    w.bad = a.take<int>(2);
    w.tst = a.take<int>(16);                                    // purification state, two parities
    w.fock = carve_fock(a, N, n_aux, n_occ, n_pairs, prec, comp);
    w.fin = fin_slab ? carve_fock(a, N, n_aux, n_occ, n_pairs, RI_FP64, true) : FockWS{};
    w.dens = carve_density(a, N, n_aux, n_pairs);
    return w;
}

// Exchange workspace layout of an SCF in precision p: with the final FP64
// build, FP32 iterations use the FP64 layout (the FP32-stored B is widened on
// load); split-BF16 iterations keep their own layout and the final build gets
// FP64 slabs of B_c.
int energy_layout(const Prec& p) { return p.fin && !is_bf16(p.base) ? RI_FP64 : p.base; }
bool energy_fin_slab(const Prec& p) { return p.fin && is_bf16(p.base); }

struct GradWS { double *D, *W, *T1, *dpair, *gamma, *c, *Bij, *Xi, *Zx, *part, *Cp, *WY; void* Xt; float* Xt32; SlabWS sw; };
GradWS carve_grad(Arena& a, int N, int n_aux, int n_occ, int64_t n_pairs, int n_centres, int prec,
                  bool comp = false) {
    GradWS w;
    w.sw = carve_slab(a, N, n_aux, prec, comp);
    const int Npad = ri::xt_ld(N);
    const int64_t n2 = (int64_t)N * N, o2 = (int64_t)n_occ * n_occ;
    w.D = a.take<double>(n2);
    w.W = a.take<double>(n2);
    w.T1 = a.take<double>(n2);
    w.dpair = a.take<double>(std::max<int64_t>(n_pairs, 1));
    w.gamma = a.take<double>(n_aux);
    w.c = a.take<double>(n_aux);
    w.Bij = a.take<double>((int64_t)n_aux * o2);
    w.Xi = a.take<double>((int64_t)n_aux * o2);
    w.Zx = a.take<double>((int64_t)n_aux * n_aux);
    w.part = a.take<double>((int64_t)(3 * ri::GRAD_BLOCKS + 1) * 3 * std::max(n_centres, 1));
    w.Cp = a.take<double>(ri::cpad_elems(N, n_occ));
    w.WY = a.take<double>((int64_t)ri::grad_slab(N, n_aux) * N * N);   // U^P C^T, one slab of P
    // X^T for B_ij, reused afterwards for U^P = C Xi^P ([n_aux][N][n_occ])
    w.Xt = a.take<char>((int64_t)n_aux * n_occ * Npad * 8 + 8);
    w.Xt32 = prec == RI_FP32 ? a.take<float>((int64_t)n_aux * n_occ * Npad) : nullptr;
    return w;
}

// One non-blocking side stream per device (default priority), created on
// first use and kept for the life of the process.
hipStream_t side_stream() {
    static std::mutex mu;
    static hipStream_t streams[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
        streams[dev] = nullptr;
    return streams[dev];
}

// Fork/join of the caller's stream with the side stream: events are made per
// call, so concurrent callers never wait on each other's records.  The
// caller's stream waits for the side stream on every exit: close() on the
// normal path, the destructor after an early error return, so no work of
// the call is left running on the side stream once the call has returned.
struct Fork {
    hipStream_t st = nullptr, side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool closed = false;
    bool open(hipStream_t s) {
        st = s;
        side = side_stream();
        if (!side || hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(fork, st) != hipSuccess || hipStreamWaitEvent(side, fork, 0) != hipSuccess) {
            side = nullptr;
            return false;
        }
        return true;
    }
    // st waits for everything enqueued on the side stream so far
    hipError_t close() {
        closed = true;
        if (!side) return hipSuccess;
        hipError_t e = hipEventRecord(join, side);
        return e == hipSuccess ? hipStreamWaitEvent(st, join, 0) : e;
    }
    ~Fork() {
        if (side && !closed) (void)close();
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
    }
};

// The Coulomb part (pair densities, gamma, J) reads only B_c and C_occ and
// is bound by HBM bandwidth; the exchange contractions are bound by MFMA
// throughput and touch none of its buffers.  The Coulomb part runs on the
// side stream, concurrently with the exchange, and the caller's stream waits
// for it before the call returns.  ev (phase-timed form): ev[0] on `st`
// before both parts, ev[1] on the side stream after the Coulomb part, ev[2]
// on `st` after X, ev[3] on `st` after the SYRK and the join (for the
// split-BF16 forms the side stream forks after X).
// With side == false everything runs on `st` (no side stream, no events): the
// same kernels and sums, so the same results bit for bit.
int32_t fock_impl(int N, int n_aux, int n_occ, const void* B, int prec, const double* Bc, const int32_t* pairs,
                  int64_t n_pairs, const double* C, double* J, double* K, double* gamma, const FockWS& w,
                  hipStream_t st, hipEvent_t* ev = nullptr, bool side = true) {
    double* g = gamma ? gamma : w.gamma;
    if (ev) HIPC(hipEventRecord(ev[0], st));
    Fork fk;
    const bool bf = is_bf16(prec);
    // The split-BF16 X holds every CU (one 141 KB-LDS workgroup each) and
    // streams B at ~4 TB/s: gamma/J beside it took longer than X itself and
    // ran on into the SYRK.  There the side stream forks after X, so
    // gamma/J runs beside the SYRK only.
    if (bf) {
        HIPC(ri::x_transform_bf16(B, prec, N, n_aux, n_occ, C, w.Cp, w.Xt, st));
        if (ev) HIPC(hipEventRecord(ev[2], st));
    }
    const bool overlap = side && fk.open(st);
    if (ev && !overlap) {
        ri::set_hip_error("side stream or its events could not be created");
        return RI_E_HIP;
    }
    // beside a large FP64 or FP32 exchange, gamma and J run on a capped grid so
    // that the X kernel's workgroups are not held back behind thousands of
    // theirs; beside the split-BF16 SYRK, which is shorter than capped gamma/J
    // would be, they keep the full grid
    const bool capped = overlap && !bf && (int64_t)n_aux * n_pairs >= ri::GJ_SIDE_MIN;
    HIPC(ri::gamma_j(Bc, pairs, n_pairs, N, n_aux, n_occ, C, w.dpair, g, w.jpart, w.js, J, overlap ? fk.side : st,
                     capped ? ri::GJ_SIDE_CAP : 0));
    if (ev) HIPC(hipEventRecord(ev[1], fk.side));
    if (bf) {
        HIPC(ri::k_syrk_bf16(w.Xt, prec, N, n_aux, n_occ, w.part, w.ks, K, st));
    } else {
        HIPC(x_any(B, prec, N, n_aux, n_occ, C, w.Cp, w.Xt, Bc, pairs, n_pairs, w.sw, st));
        if (ev) HIPC(hipEventRecord(ev[2], st));
        HIPC(ri::k_syrk(w.Xt, prec, N, n_aux, n_occ, w.part, w.ks, K, st));
    }
    HIPC(fk.close());
    if (ev) HIPC(hipEventRecord(ev[3], st));
    return RI_OK;
}

// Occupied orbitals of the Fock matrix Fx (the n_occ lowest solutions of
// F C = S C eps): projector by TC2 purification in the basis orthonormalised
// by L_S^{-1}, then an orthonormal basis of its range by two passes of
// projection and Cholesky QR, mapped back by L_S^{-T}.  The purification
// steps are launched in chunks (first `pred` steps, the previous
// purification's count plus two, then 8 at a time) and the state is read once
// per chunk; steps after the last one exit at once.
int32_t occupied_space(const double* Fx, int N, int n_occ, EnergyWS& w, bool have_prev, double* C_out,
                       int max_it, int& pred, hipStream_t st) {
    const int64_t n2 = (int64_t)N * N;
    // L_S^{-1} F L_S^{-T}, skipping the zero triangle of L_S^{-1} in both products
    HIPC(ri::gemm_f64(false, false, N, N, N, 1.0, w.LinvS, N, 0, Fx, N, 0, 0.0, w.T1, N, 0, 1, 1, 0, st));
    HIPC(ri::gemm_f64(false, true, N, N, N, 1.0, w.T1, N, 0, w.LinvS, N, 0, 0.0, w.T2, N, 0, 1, 3, 0, st));
    HIPC(ri::gershgorin(w.T2, N, w.scal + 16, w.red, st));
    const int tiles = ri::tc2f_tiles(N);
    HIPC(ri::tc2f_init(w.T2, w.scal + 16, N, w.X, w.tpart, w.tst, st));
    int k = 0, chunk = std::max(8, std::min(pred, max_it)), hs[8] = {};
    while (true) {
        const int upto = std::min(max_it, k + chunk);
        for (; k < upto; ++k) {
            const int p = k & 1;
            HIPC(ri::tc2f_step(p ? w.X2 : w.X, p ? w.X : w.X2, N, n_occ, w.tpart + 2 * tiles * p,
                               w.tpart + 2 * tiles * (p ^ 1), w.tst + 8 * p, w.tst + 8 * (p ^ 1), p ? 0 : 1, st));
        }
        HIPC(hipMemcpyAsync(hs, w.tst + 8 * (k & 1), sizeof(hs), hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        if (hs[1] || k >= max_it) break;
        chunk = 8;
    }
    // a projector that reached the idempotency threshold is used even when the
    // step limit cut its last extra steps short
    if (hs[0] < 0) return RI_E_NO_PURIFY;
    pred = hs[2] + 2;
    HIPC(ri::tc2f_final(w.X, w.X2, N, w.tst + 8 * (k & 1), st));
    if (!have_prev) HIPC(ri::hash_matrix(w.Cp, (int64_t)N * n_occ, 0x5eed1234u, st));
    for (int pass = 0; pass < 2; ++pass) {
        HIPC(ri::gemm_f64(false, false, N, n_occ, N, 1.0, w.X, N, 0, w.Cp, n_occ, 0, 0.0, w.Y, n_occ, 0, 1, 0, 0, st));
        HIPC(ri::gemm_f64(true, false, n_occ, n_occ, N, 1.0, w.Y, n_occ, 0, w.Y, n_occ, 0, 0.0, w.Mo, n_occ, 0, 1, 0,
                          0, st));
        HIPC(ri::cholesky_inv(w.Mo, n_occ, n_occ, w.LinvM, n_occ, w.dinvM, w.bad + 1, st));
        HIPC(ri::gemm_f64(false, true, N, n_occ, n_occ, 1.0, w.Y, n_occ, 0, w.LinvM, n_occ, 0, 0.0, w.Cp, n_occ, 0,
                          1, 0, 0, st));
    }
    HIPC(ri::gemm_f64(true, false, N, n_occ, N, 1.0, w.LinvS, N, 0, w.Cp, n_occ, 0, 0.0, C_out, n_occ, 0, 1, 2, 0,
                      st));
    return RI_OK;
}

// Scratch of ri_fock_jk_noalloc: a static device array, one copy on each
// device the library runs on, held until the process ends.  Host code never
// names it except to look up its device address.
static __device__ __align__(256) char scratch[RI_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int32_t noalloc_scratch(void** out) {
    static std::mutex mu;
    static void* ptrs[64] = {};
    int dev = 0;
    HIPC(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return RI_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptrs[dev]) {
        void* p = nullptr;
        HIPC(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        ptrs[dev] = p;
    }
    *out = ptrs[dev];
    return RI_OK;
}

}  // namespace

namespace ri {
void set_hip_error(const char* text) { g_hip_err = text; }
}  // namespace ri

extern "C" {

const char* ri_version(void) { return "libri 0.1 (gfx950)"; }

const char* ri_last_hip_error(void) { return g_hip_err.c_str(); }

const char* ri_status_str(int32_t s) {
    switch (s) {
        case RI_OK: return "ok";
        case RI_E_ARG: return "invalid argument";
        case RI_E_NOT_PD: return "matrix not positive definite";
        case RI_E_NO_CONV: return "iteration did not converge";
        case RI_E_WORKSPACE: return "workspace too small";
        case RI_E_CAPACITY: return "pair capacity too small";
        case RI_E_HIP: return "HIP runtime error";
        case RI_E_UNSUPPORTED: return "unsupported option";
        case RI_E_NO_PURIFY: return "purification did not reach an idempotent projector";
        default: return "unknown status";
    }
}

size_t ri_packed_b_bytes(int32_t N, int32_t n_aux, int32_t prec) {
    if (N <= 0 || n_aux <= 0 || prec < 0 || prec > 3) return 0;
    if (is_bf16(prec)) {
        const int64_t nt = ri::n_tiles_1d(N);
        return (size_t)ri::bf16_parts(prec) * n_aux * nt * nt * 4096 * 2;
    }
    return (size_t)n_aux * ri::tile_elems(N) * elem_size(prec);
}

size_t ri_workspace_bytes(int32_t op, int32_t N, int32_t n_aux, int32_t n_occ, int64_t n_pairs, int32_t prec_arg) {
    const Prec pp = split_prec(prec_arg, op == RI_OP_ENERGY);
    const int prec = pp.base;
    if (N <= 0 || n_aux <= 0 || n_occ <= 0 || n_pairs < 0 || !pp.ok) return 0;
    Arena a{nullptr, 0, 0, true};
    switch (op) {
        case RI_OP_BUILD_3C: carve_build(a, N); break;
        case RI_OP_METRIC: carve_metric(a, N, n_aux, n_pairs); break;
        case RI_OP_FOCK: carve_fock(a, N, n_aux, n_occ, n_pairs, prec, pp.comp); break;
        case RI_OP_ENERGY:
            carve_energy(a, N, n_aux, n_occ, n_pairs, energy_layout(pp), 8, pp.comp, energy_fin_slab(pp));
            break;
        case RI_OP_GRADIENT:
            carve_grad(a, N, n_aux, n_occ, n_pairs, 2048, is_bf16(prec) ? RI_FP64 : prec, pp.comp || is_bf16(prec));
            break;
        case RI_OP_FOCK_DENSITY: carve_density(a, N, n_aux, n_pairs); break;
        case RI_OP_MLP: {
            size_t off = 0;
            ri::carve_mlp(nullptr, 0, off, std::max<int64_t>(n_pairs, 1));
            return off + 256;
        }
        default: return 0;
    }
    return a.off + 256;
}

int32_t ri_build_3c(const ri_system* sys, double tau, int32_t* pairs, int64_t cap, int64_t* n_pairs, double* T,
                    void* ws, size_t ws_bytes, hipStream_t st) {
    if (!valid_sys(sys) || !pairs || !n_pairs || cap < 0 || !ws || !(tau >= 0.0)) return RI_E_ARG;
    Arena a{(char*)ws, ws_bytes, 0, false};
    BuildWS w = carve_build(a, sys->n_fn);
    if (!a.ok()) return RI_E_WORKSPACE;
    HIPC(ri::screen_pairs(sys, tau, w.counts, w.offsets, st));
    int64_t np = 0;
    HIPC(hipMemcpyAsync(&np, w.offsets + sys->n_fn, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    *n_pairs = np;
    if (np > cap) return RI_E_CAPACITY;
    HIPC(ri::write_pairs(sys, tau, w.offsets, pairs, st));
    if (T) HIPC(ri::eri3(sys, pairs, np, T, st));
    return RI_OK;
}

int32_t ri_metric_factor(const ri_system* sys, const int32_t* pairs, int64_t n_pairs, double* T, double* L,
                         double* Linv, void* B, int32_t prec_arg, int64_t* bad_pivot, void* ws, size_t ws_bytes,
                         hipStream_t st) {
    if (!valid_sys(sys) || n_pairs < 0 || (n_pairs > 0 && (!pairs || !T)) || !L || !Linv || !bad_pivot || !ws)
        return RI_E_ARG;
    const Prec pp = split_prec(prec_arg);
    if (!pp.ok) return RI_E_UNSUPPORTED;
    const int prec = pp.base;
    const int na = sys->n_aux, N = sys->n_fn;
    Arena a{(char*)ws, ws_bytes, 0, false};
    MetricWS w = carve_metric(a, N, na, n_pairs);
    if (!a.ok()) return RI_E_WORKSPACE;
    *bad_pivot = -1;
    // L^{-1} and the packing of each block of B rows run on the side stream:
    // each block step of L^{-1} as soon as the Cholesky has made its block
    // column final (beside the chain of diagonal factorisations, which keeps
    // only a few CUs busy), each packing once the triangular solve has
    // finished its rows (the solve is bound by MFMA throughput, the packing
    // by memory bandwidth).  Small problems keep one stream: many callers'
    // setups, as the batched workload's, would otherwise share the one side
    // stream.
    struct Events {
        std::vector<hipEvent_t> e;
        ~Events() {
            for (hipEvent_t x : e) (void)hipEventDestroy(x);
        }
    } evs;
    HIPC(ri::metric(sys, L, st));
    HIPC(ri::fill_i32(w.bad, INT_MAX, 1, st));
    Fork fk;
    const bool side = (int64_t)na * n_pairs >= ri::GJ_SIDE_MIN && fk.open(st);
    hipStream_t ss = side ? fk.side : st;
    // the side stream waits for everything enqueued on st so far
    auto side_waits = [&]() -> hipError_t {
        if (!side) return hipSuccess;
        hipEvent_t e = nullptr;
        RI_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        evs.e.push_back(e);
        RI_TRY(hipEventRecord(e, st));
        return hipStreamWaitEvent(ss, e, 0);
    };
    HIPC(ri::tri_inverse_begin(Linv, na, na, ss));
    auto inverse_step = [&](int k) -> hipError_t {
        RI_TRY(side_waits());
        return ri::tri_inverse_steps(L, na, na, w.dinv, Linv, na, k, k + 1, ss);
    };
    HIPC(ri::cholesky_inv(L, na, na, nullptr, na, w.dinv, w.bad, st, inverse_step));
    int bad = INT_MAX;
    HIPC(hipMemcpyAsync(&bad, w.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (bad != INT_MAX) {
        *bad_pivot = bad;
        return RI_E_NOT_PD;
    }
    if (B) HIPC(ri::pair_map(pairs, n_pairs, N, w.map, st));
    const int64_t b_row = B ? (int64_t)ri_packed_b_bytes(N, 1, prec) : 0;   // bytes of one auxiliary's packed tiles
    auto pack_rows = [&](int r0, int r1) -> hipError_t {
        if (!B) return hipSuccess;
        RI_TRY(side_waits());
        const double* rows = T + (int64_t)r0 * n_pairs;
        void* out = (char*)B + r0 * b_row;
        return is_bf16(prec) ? ri::pack_b_bf16(rows, n_pairs, w.map, N, r1 - r0, out, prec, ss)
                             : ri::pack_b(rows, n_pairs, w.map, N, r1 - r0, out, prec, ss);
    };
    // Bc = L^{-1} T by recursive blocked forward substitution, in place over T.
    if (n_pairs > 0) {
        HIPC(ri::trsm_band(L, na, na, w.dinv, w.band, st));
        HIPC(ri::trsm_rec(L, na, na, w.band, T, (int)n_pairs, n_pairs, st, 0, pack_rows));
    } else {
        HIPC(pack_rows(0, na));
    }
    HIPC(fk.close());
    return RI_OK;
}

int32_t ri_pack_b(int32_t N, int32_t n_aux, const double* Bc, const int32_t* pairs, int64_t n_pairs, void* B,
                  int32_t prec, void* ws, size_t ws_bytes, hipStream_t st) {
    if (N <= 0 || n_aux <= 0 || n_pairs < 0 || (n_pairs > 0 && (!Bc || !pairs)) || !B || !ws) return RI_E_ARG;
    if (prec != RI_FP64 && prec != RI_FP32 && !is_bf16(prec)) return RI_E_UNSUPPORTED;
    Arena a{(char*)ws, ws_bytes, 0, false};
    MetricWS w = carve_metric(a, N, n_aux, n_pairs);
    if (!a.ok()) return RI_E_WORKSPACE;
    HIPC(ri::pair_map(pairs, n_pairs, N, w.map, st));
    if (is_bf16(prec)) HIPC(ri::pack_b_bf16(Bc, n_pairs, w.map, N, n_aux, B, prec, st));
    else HIPC(ri::pack_b(Bc, n_pairs, w.map, N, n_aux, B, prec, st));
    return RI_OK;
}

int32_t ri_fock_jk(int32_t N, int32_t n_aux, int32_t n_occ, const void* B, int32_t prec_arg, const double* Bc,
                   const int32_t* pairs, int64_t n_pairs, const double* C, double* J, double* K, double* gamma,
                   void* ws, size_t ws_bytes, hipStream_t st) {
    const Prec pp = split_prec(prec_arg);
    const int prec = pp.base;
    if (N <= 0 || n_aux <= 0 || n_occ <= 0 || n_occ > N || n_pairs < 0 || (!B && !pp.comp) || !C || !J || !K ||
        !ws || (n_pairs > 0 && (!Bc || !pairs)))
        return RI_E_ARG;
    if (!pp.ok || (is_bf16(prec) && n_occ > 128)) return RI_E_UNSUPPORTED;
    if (pp.comp) B = nullptr;
    Arena a{(char*)ws, ws_bytes, 0, false};
    FockWS w = carve_fock(a, N, n_aux, n_occ, n_pairs, prec, pp.comp);
    if (!a.ok()) return RI_E_WORKSPACE;
    return fock_impl(N, n_aux, n_occ, B, prec, Bc, pairs, n_pairs, C, J, K, gamma, w, st);
}

int32_t ri_fock_jk_noalloc(int32_t N, int32_t n_aux, int32_t n_occ, const void* B, int32_t prec_arg,
                           const double* Bc, const int32_t* pairs, int64_t n_pairs, const double* C, double* J,
                           double* K, double* gamma, hipStream_t st) {
    const Prec pp = split_prec(prec_arg);
    const int prec = pp.base;
    if (N <= 0 || n_aux <= 0 || n_occ <= 0 || n_occ > N || n_pairs < 0 || (!B && !pp.comp) || !C || !J || !K ||
        (n_pairs > 0 && (!Bc || !pairs)))
        return RI_E_ARG;
    if (!pp.ok || (is_bf16(prec) && n_occ > 128)) return RI_E_UNSUPPORTED;
    if (pp.comp) B = nullptr;
    Arena dry{nullptr, 0, 0, true};
    carve_fock(dry, N, n_aux, n_occ, n_pairs, prec, pp.comp);
    if (dry.off + 256 > RI_NOALLOC_SCRATCH_BYTES) return RI_E_WORKSPACE;
    void* ws = nullptr;
    const int32_t rc = noalloc_scratch(&ws);
    if (rc != RI_OK) return rc;
    Arena a{(char*)ws, RI_NOALLOC_SCRATCH_BYTES, 0, false};
    FockWS w = carve_fock(a, N, n_aux, n_occ, n_pairs, prec, pp.comp);
    return fock_impl(N, n_aux, n_occ, B, prec, Bc, pairs, n_pairs, C, J, K, gamma, w, st, nullptr, false);
}

int32_t ri_fock_jk_timed(int32_t N, int32_t n_aux, int32_t n_occ, const void* B, int32_t prec_arg,
                         const double* Bc, const int32_t* pairs, int64_t n_pairs, const double* C, double* J,
                         double* K, double* gamma, void* ws, size_t ws_bytes, hipStream_t st, hipEvent_t* events) {
    if (!events || !events[0] || !events[1] || !events[2] || !events[3]) return RI_E_ARG;
    const Prec pp = split_prec(prec_arg);
    const int prec = pp.base;
    if (N <= 0 || n_aux <= 0 || n_occ <= 0 || n_occ > N || n_pairs < 0 || (!B && !pp.comp) || !C || !J || !K ||
        !ws || (n_pairs > 0 && (!Bc || !pairs)))
        return RI_E_ARG;
    if (!pp.ok || (is_bf16(prec) && n_occ > 128)) return RI_E_UNSUPPORTED;
    if (pp.comp) B = nullptr;
    Arena a{(char*)ws, ws_bytes, 0, false};
    FockWS w = carve_fock(a, N, n_aux, n_occ, n_pairs, prec, pp.comp);
    if (!a.ok()) return RI_E_WORKSPACE;
    return fock_impl(N, n_aux, n_occ, B, prec, Bc, pairs, n_pairs, C, J, K, gamma, w, st, events);
}

int32_t ri_fock_jk_density(int32_t N, int32_t n_aux, const double* Bc, const int32_t* pairs, int64_t n_pairs,
                           const double* D, double* J, double* K, double* gamma, void* ws, size_t ws_bytes,
                           hipStream_t st) {
    if (N <= 0 || n_aux <= 0 || n_pairs < 0 || !D || !J || !K || !ws || (n_pairs > 0 && (!Bc || !pairs)))
        return RI_E_ARG;
    Arena a{(char*)ws, ws_bytes, 0, false};
    DensityWS w = carve_density(a, N, n_aux, n_pairs);
    if (!a.ok()) return RI_E_WORKSPACE;
    HIPC(jk_density(Bc, pairs, n_pairs, N, n_aux, D, J, K, gamma, w, st));
    return RI_OK;
}

int32_t ri_energy(const ri_system* sys, const void* B, int32_t prec_arg, const double* Bc, const int32_t* pairs,
                  int64_t n_pairs, const ri_scf_opts* opts, const double* guess, double* C_occ, double* F_out,
                  double* D_out, ri_scf_result* res, void* ws, size_t ws_bytes, hipStream_t st) {
    const Prec pp = split_prec(prec_arg, true);
    const int prec = pp.base;
    if (!valid_sys(sys) || (!B && !pp.comp) || !opts || !C_occ || !F_out || !res || !ws || n_pairs < 0 ||
        (n_pairs > 0 && (!Bc || !pairs)))
        return RI_E_ARG;
    if (pp.comp) B = nullptr;
    if (opts->diis_n < 1 || opts->diis_n > 8 || opts->max_iter < 1 || !(opts->tol_E > 0) || !(opts->tol_err > 0))
        return RI_E_ARG;
    if (opts->guess_kind != 0 && !guess) return RI_E_ARG;
    if (opts->max_purify < 0) return RI_E_ARG;
    const int npur = opts->max_purify > 0 ? opts->max_purify : 200;
    int pred = 40;   // purification steps launched before the first state read
    if (opts->guess_kind < 0 || opts->guess_kind > 3) return RI_E_UNSUPPORTED;
    if (!pp.ok || (is_bf16(prec) && sys->n_occ > 128)) return RI_E_UNSUPPORTED;
    // Two bfloat16 parts hold B and C_occ to about 2^-17: at the 8-centre
    // workload that rounding alone moves the energy by 1.6e-6 Eh (B) and
    // 8e-6 Eh (C_occ), and the SYRK's dropped lo x lo product is a Gram matrix,
    // so its error does not cancel.  BF16X3 iterations are therefore offered
    // only with the final FP64 exchange build, which removes them to first order.
    if (prec == RI_BF16X3 && !pp.fin) return RI_E_UNSUPPORTED;
    const int N = sys->n_fn, na = sys->n_aux, no = sys->n_occ, dn = opts->diis_n;
    const int64_t n2 = (int64_t)N * N;
    Arena a{(char*)ws, ws_bytes, 0, false};
    EnergyWS w = carve_energy(a, N, na, no, n_pairs, energy_layout(pp), 8, pp.comp, energy_fin_slab(pp));
    if (!a.ok()) return RI_E_WORKSPACE;
    std::memset(res, 0, sizeof(*res));

    HIPC(ri::one_electron(sys, w.S, w.H, st));
    HIPC(ri::nuclear_repulsion(sys, w.scal + 8, st));
    HIPC(ri::copy(w.Ls, w.S, n2, st));
    HIPC(ri::fill_i32(w.bad, INT_MAX, 2, st));
    HIPC(ri::cholesky_inv(w.Ls, N, N, w.LinvS, N, w.dinvS, w.bad, st));
    int bad = INT_MAX;
    HIPC(hipMemcpyAsync(&bad, w.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (bad != INT_MAX) return RI_E_NOT_PD;

    int32_t rc;
    if (opts->guess_kind == 0) {
        rc = occupied_space(w.H, N, no, w, false, C_occ, npur, pred, st);
        if (rc) return rc;
    } else if (opts->guess_kind == 3) {
        // Fock matrix of the density itself (J and K from D), then its occupied space
        HIPC(jk_density(Bc, pairs, n_pairs, N, na, guess, w.J, w.K, nullptr, w.dens, st));
        HIPC(ri::fock_assemble(w.H, w.J, w.K, w.F, n2, st));
        rc = occupied_space(w.F, N, no, w, false, C_occ, npur, pred, st);
        if (rc) return rc;
    } else if (opts->guess_kind == 2) {
        // occupied space of the density: lowest solutions of (-S D S) v = l S v
        HIPC(ri::gemm_f64(false, false, N, N, N, 1.0, w.S, N, 0, guess, N, 0, 0.0, w.T1, N, 0, 1, 0, 0, st));
        HIPC(ri::gemm_f64(false, false, N, N, N, -1.0, w.T1, N, 0, w.S, N, 0, 0.0, w.Fx, N, 0, 1, 0, 0, st));
        rc = occupied_space(w.Fx, N, no, w, false, C_occ, npur, pred, st);
        if (rc) return rc;
    } else {
        HIPC(ri::copy(C_occ, guess, (int64_t)N * no, st));
        // the guess in the orthonormal frame, C' = L_S^T C, seeds the subspace passes
        HIPC(ri::gemm_f64(true, false, N, no, N, 1.0, w.Ls, N, 0, C_occ, no, 0, 0.0, w.Cp, no, 0, 1, 2, 0, st));
    }

    std::vector<int> slots;
    HIPC(ri::fill(w.Bfull, 0.0, 64, st));   // DIIS inner products <e_i, e_j>, indexed by ring slot
    int pushes = 0;
    double E_old = 0.0, host[8];
    bool converged = false;
    int it = 0;
    for (it = 1; it <= opts->max_iter; ++it) {
        rc = fock_impl(N, na, no, B, prec, Bc, pairs, n_pairs, C_occ, w.J, w.K, nullptr, w.fock, st);
        if (rc) return rc;
        HIPC(ri::fock_assemble(w.H, w.J, w.K, w.F, n2, st));
        HIPC(ri::gemm_f64(false, true, N, N, no, 2.0, C_occ, no, 0, C_occ, no, 0, 0.0, w.D, N, 0, 1, 0, 0, st));
        HIPC(ri::energy_terms(w.D, w.H, w.J, w.K, n2, w.scal + 8, w.scal, w.red, st));
        HIPC(ri::gemm_f64(false, false, N, N, N, 1.0, w.F, N, 0, w.D, N, 0, 0.0, w.T1, N, 0, 1, 0, 0, st));
        HIPC(ri::gemm_f64(false, false, N, N, N, 1.0, w.T1, N, 0, w.S, N, 0, 0.0, w.T2, N, 0, 1, 0, 0, st));
        HIPC(ri::commutator(w.T2, w.E, N, st));
        HIPC(ri::max_abs(w.E, n2, w.scal + 5, w.red, st));
        HIPC(hipMemcpyAsync(host, w.scal, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        res->E_total = host[0];
        res->E_nuc = host[1];
        res->E_1e = host[2];
        res->E_J = host[3];
        res->E_K = host[4];
        res->max_err = host[5];
        res->n_iter = it;
        if (it > 1) {
            res->last_dE = host[0] - E_old;
            if (std::fabs(host[0] - E_old) < opts->tol_E && host[5] < opts->tol_err) {
                converged = true;
                break;
            }
        }
        E_old = host[0];
        // DIIS: store (F, e) in the ring, update the B matrix row, extrapolate.
        const int s = pushes % dn;
        ++pushes;
        HIPC(ri::copy(w.dF[s], w.F, n2, st));
        HIPC(ri::copy(w.dE[s], w.E, n2, st));
        for (size_t k = 0; k < slots.size(); ++k)
            if (slots[k] == s) { slots.erase(slots.begin() + k); break; }
        slots.push_back(s);
        const int m = (int)slots.size();
        {
            const double* es[8];
            for (int k = 0; k < m; ++k) es[k] = w.dE[slots[k]];
            HIPC(ri::diis_dots(es, m, w.dE[s], w.row, n2, w.red, st));
            HIPC(ri::diis_prep(w.Bfull, w.row, slots.data(), m, s, w.Bmat, st));
        }
        const double* Fx = w.F;
        if (m >= 2) {
            const double* fs[8];
            for (int k = 0; k < m; ++k) fs[k] = w.dF[slots[k]];
            HIPC(ri::diis_solve(w.Bmat, m, 8, w.coef, st));
            HIPC(ri::diis_combine(fs, w.coef, m, w.Fx, n2, st));
            Fx = w.Fx;
        }
        rc = occupied_space(Fx, N, no, w, true, C_occ, npur, pred, st);
        if (rc) return rc;
    }
    if (pp.fin && converged) {
        // one exchange build in FP64 arithmetic at the converged density: from
        // the FP32-stored B widened on load, or (split-BF16 forms, whose parts
        // hold B only to 2^-17 or 2^-25) from the FP64 B_c unpacked slab by
        // slab; the energy from the same D, h and J
        if (is_bf16(prec)) {
            HIPC(x_any(nullptr, RI_FP64, N, na, no, C_occ, w.fin.Cp, w.fin.Xt, Bc, pairs, n_pairs, w.fin.sw, st));
            HIPC(ri::k_syrk(w.fin.Xt, RI_FP64, N, na, no, w.fin.part, w.fin.ks, w.K, st));
        } else {
            HIPC(ri::x_transform(B, ri::X_F64_B32, N, na, no, C_occ, w.fock.Cp, w.fock.Xt, st));
            HIPC(ri::k_syrk(w.fock.Xt, RI_FP64, N, na, no, w.fock.part, w.fock.ks, w.K, st));
        }
        HIPC(ri::energy_terms(w.D, w.H, w.J, w.K, n2, w.scal + 8, w.scal, w.red, st));
        HIPC(hipMemcpyAsync(host, w.scal, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        res->E_total = host[0];
        res->E_1e = host[2];
        res->E_J = host[3];
        res->E_K = host[4];
    }
    HIPC(ri::copy(F_out, w.F, n2, st));
    if (D_out) HIPC(ri::copy(D_out, w.D, n2, st));
    HIPC(hipStreamSynchronize(st));
    res->converged = converged ? 1 : 0;
    return converged ? RI_OK : RI_E_NO_CONV;
}

int32_t ri_gradient(const ri_system* sys, const int32_t* pairs, int64_t n_pairs, const void* B, int32_t prec_arg,
                    const double* Bc, const double* Linv, const double* C, const double* F, double* grad, void* ws,
                    size_t ws_bytes, hipStream_t st) {
    const Prec pp = split_prec(prec_arg);
    // The split-BF16 forms form B_ij^P = C^T B^P C in FP64 arithmetic from B_c,
    // slab by slab as the compressed form does: Xi and Z enter the gradient
    // linearly, and their parts would carry B's 2^-17 (or 2^-25) rounding.
    const bool slabs = pp.comp || is_bf16(pp.base);
    const int prec = is_bf16(pp.base) ? RI_FP64 : pp.base;
    if (!valid_sys(sys) || (!B && !slabs) || !Linv || !C || !F || !grad || !ws || n_pairs < 0 ||
        (n_pairs > 0 && (!Bc || !pairs)))
        return RI_E_ARG;
    if (!pp.ok) return RI_E_UNSUPPORTED;
    if (slabs) B = nullptr;
    if (sys->n_centres > 2048) return RI_E_UNSUPPORTED;
    const int N = sys->n_fn, na = sys->n_aux, no = sys->n_occ, nc = sys->n_centres;
    const int Npad = ri::xt_ld(N);
    const int64_t o2 = (int64_t)no * no;
    Arena a{(char*)ws, ws_bytes, 0, false};
    GradWS w = carve_grad(a, N, na, no, n_pairs, 2048, prec, slabs);
    if (!a.ok()) return RI_E_WORKSPACE;
    // D = 2 C C^T, W = 1/2 D F D
    HIPC(ri::gemm_f64(false, true, N, N, no, 2.0, C, no, 0, C, no, 0, 0.0, w.D, N, 0, 1, 0, 0, st));
    HIPC(ri::gemm_f64(false, false, N, N, N, 1.0, F, N, 0, w.D, N, 0, 0.0, w.T1, N, 0, 1, 0, 0, st));
    HIPC(ri::gemm_f64(false, false, N, N, N, 0.5, w.D, N, 0, w.T1, N, 0, 0.0, w.W, N, 0, 1, 0, 0, st));
    const int GB = ri::GRAD_BLOCKS;
    const int64_t rowlen = 3 * (int64_t)nc;
    // On the side stream, beside X and the exchange products (they share no
    // buffers): gamma = L^{-1} d, c = L^{-T} gamma = A^{-1} d and the
    // one-electron term.  Without a side stream they run here in turn.
    Fork fk;
    hipStream_t ss = fk.open(st) ? fk.side : st;
    HIPC(ri::gamma_only(Bc, pairs, n_pairs, na, no, C, w.dpair, w.gamma, ss));
    HIPC(ri::gemm_f64(true, false, na, 1, na, 1.0, Linv, na, 0, w.gamma, 1, 0, 0.0, w.c, 1, 0, 1, 2, 0, ss));
    HIPC(ri::grad_one_electron(sys, w.D, w.W, w.part, ss));
    // B_ij^P = (C^T B^P C)_ij from X^P = B^P C
    if (prec == RI_FP32) {
        HIPC(x_any(B, prec, N, na, no, C, w.Cp, w.Xt32, Bc, pairs, n_pairs, w.sw, st));
        HIPC(ri::widen(w.Xt32, (double*)w.Xt, (int64_t)na * no * Npad, st));
    } else {
        HIPC(x_any(B, prec, N, na, no, C, w.Cp, w.Xt, Bc, pairs, n_pairs, w.sw, st));
    }
    // one GEMM over all (P, i) rows: the rows of X^T are stacked P-major, as B_ij's
    HIPC(ri::gemm_f64(false, false, na * no, no, N, 1.0, (const double*)w.Xt, Npad, 0, C, no, 0, 0.0, w.Bij, no, 0,
                      1, 0, 0, st, 128));
    // Xi = L^{-T} B_ij  (columns ij)
    HIPC(ri::gemm_f64(true, false, na, (int)o2, na, 1.0, Linv, na, 0, w.Bij, o2, 0, 0.0, w.Xi, o2, 0, 1, 2, 0, st));
    // Zx = -2 sum_ij Xi_ij Xi_ij^T (lower tiles); Z = c c^T + Zx inside the contraction
    HIPC(ri::grad_metric_z(w.Xi, na, o2, w.WY, (int64_t)ri::grad_slab(N, na) * N * N, w.Zx, st));
    // U^P = C Xi^P  (stored over the X buffer)
    double* U = (double*)w.Xt;
    HIPC(ri::u_products(C, w.Xi, N, no, na, U, st));
    HIPC(fk.close());   // c and the one-electron rows are ready on st from here
    HIPC(ri::grad_metric(sys, w.Zx, w.c, w.part + GB * rowlen, st));
    HIPC(ri::grad_three_centre(sys, pairs, n_pairs, U, C, no, w.D, w.c, w.WY, w.part + 2 * GB * rowlen, st));
    HIPC(ri::grad_nuclear(sys, w.part + 3 * GB * rowlen, st));
    HIPC(ri::grad_reduce(w.part, 3 * GB + 1, nc, grad, st));
    return RI_OK;
}

int32_t ri_pair_features(const ri_system* sys, const int32_t* pairs, int64_t n_pairs, float* feat, hipStream_t st) {
    if (!valid_sys(sys) || n_pairs < 0 || (n_pairs > 0 && (!pairs || !feat))) return RI_E_ARG;
    HIPC(ri::pair_features(sys, pairs, n_pairs, feat, st));
    return RI_OK;
}

static bool valid_mlp(const ri_mlp* net) { return net && net->params && net->mu && net->sigma; }

int32_t ri_mlp_forward(const ri_mlp* net, const float* feat, int64_t n, float* y, int32_t prec, void* ws,
                       size_t ws_bytes, hipStream_t st) {
    if (!valid_mlp(net) || n <= 0 || !feat || !y || !ws) return RI_E_ARG;
    if (prec != RI_MLP_FP32 && prec != RI_MLP_BF16) return RI_E_UNSUPPORTED;
    size_t off = 0;
    ri::carve_mlp(nullptr, 0, off, n);
    if (off + 256 > ws_bytes) return RI_E_WORKSPACE;
    off = 0;
    ri::MlpWS w = ri::carve_mlp((char*)ws, ws_bytes, off, n);
    HIPC(ri::mlp_forward(net, feat, n, y, prec, w, st));
    return RI_OK;
}

int32_t ri_mlp_train_step(const ri_mlp* net, float* m, float* v, int32_t step, float lr, const float* feat,
                          const float* target, int64_t n, float* loss, float* grad, void* ws, size_t ws_bytes,
                          hipStream_t st) {
    if (!valid_mlp(net) || !m || !v || step < 1 || !(lr > 0.0f) || n <= 0 || !feat || !target || !loss || !ws)
        return RI_E_ARG;
    size_t off = 0;
    ri::carve_mlp(nullptr, 0, off, n);
    if (off + 256 > ws_bytes) return RI_E_WORKSPACE;
    off = 0;
    ri::MlpWS w = ri::carve_mlp((char*)ws, ws_bytes, off, n);
    HIPC(ri::mlp_train_step(net, m, v, step, lr, feat, target, n, loss, w, st));
    if (grad) HIPC(hipMemcpyAsync(grad, w.grad, sizeof(float) * RI_MLP_NPARAM, hipMemcpyDeviceToDevice, st));
    return RI_OK;
}

int32_t ri_density_from_pairs(int32_t N, const int32_t* pairs, int64_t n_pairs, const float* d, double* D,
                              hipStream_t st) {
    if (N <= 0 || n_pairs < 0 || !D || (n_pairs > 0 && (!pairs || !d))) return RI_E_ARG;
    HIPC(ri::scatter_density(N, pairs, n_pairs, d, D, st));
    return RI_OK;
}

int32_t ri_density_to_pairs(int32_t N, const int32_t* pairs, int64_t n_pairs, const double* D, float* d,
                            hipStream_t st) {
    if (N <= 0 || n_pairs < 0 || !D || (n_pairs > 0 && (!pairs || !d))) return RI_E_ARG;
    HIPC(ri::gather_density(N, pairs, n_pairs, D, d, st));
    return RI_OK;
}

int32_t ri_pair_delta_features(const ri_system* sys, const double* xyz_prev, const int32_t* pairs, int64_t n_pairs,
                               const double* D_prev, float* feat, hipStream_t st) {
    if (!valid_sys(sys) || !xyz_prev || !D_prev || n_pairs < 0 || (n_pairs > 0 && (!pairs || !feat))) return RI_E_ARG;
    HIPC(ri::pair_delta_features(sys, xyz_prev, pairs, n_pairs, D_prev, feat, st));
    return RI_OK;
}

int32_t ri_density_change_pairs(int32_t N, const int32_t* pairs, int64_t n_pairs, const double* D_new,
                                const double* D_prev, float scale, float* d, hipStream_t st) {
    if (N <= 0 || n_pairs < 0 || !D_new || !D_prev || (n_pairs > 0 && (!pairs || !d))) return RI_E_ARG;
    HIPC(ri::density_change(N, pairs, n_pairs, D_new, D_prev, scale, d, st));
    return RI_OK;
}

int32_t ri_density_add_pairs(int32_t N, const int32_t* pairs, int64_t n_pairs, const float* d, double scale,
                             const double* D_prev, double* D_out, hipStream_t st) {
    if (N <= 0 || n_pairs < 0 || !D_prev || !D_out || D_prev == D_out || (n_pairs > 0 && (!pairs || !d)))
        return RI_E_ARG;
    HIPC(ri::density_add(N, pairs, n_pairs, d, scale, D_prev, D_out, st));
    return RI_OK;
}

}  // extern "C"
