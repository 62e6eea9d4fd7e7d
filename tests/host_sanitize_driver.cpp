// Host-layer checks of libri under AddressSanitizer and UBSan.
//
// Linked with every libri source, whose host code is built with both
// sanitizers, and run on a machine without a GPU (a kernel launch there fails
// with a HIP error).  It drives every host path that decides something
// before or without device work: workspace layouts of every operation and
// precision (including the batched plan), argument and option validation,
// the workspace-size contract, and the RI_E_HIP path of a call that reaches
// the runtime.  Any sanitizer report aborts the run; a wrong status exits 1.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../include/ri.h"

static int failures = 0;
#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

int main() {
    // every status has text
    for (int c = 0; c <= 9; ++c) EXPECT(ri_status_str(c) && std::strlen(ri_status_str(c)) > 0);
    EXPECT(std::strlen(ri_version()) > 0);

    // workspace layouts over a grid of shapes, operations and precision arguments
    const int precs[] = {RI_FP64, RI_FP32, RI_BF16X3, RI_BF16X6, RI_FP64 | RI_COMPRESSED, RI_FP32 | RI_COMPRESSED,
                         RI_FP32 | RI_FINAL_FP64, RI_BF16X3 | RI_FINAL_FP64, RI_BF16X6 | RI_FINAL_FP64,
                         RI_FP64 | RI_FINAL_FP64, RI_BF16X6 | RI_COMPRESSED, 4, -1, 0x7f};
    const int shapes[][3] = {{1, 1, 1}, {32, 80, 8}, {63, 64, 1}, {64, 65, 64}, {129, 300, 100}, {1000, 3000, 100},
                             {4096, 12000, 500}};
    for (auto& sh : shapes)
        for (int op = 0; op <= 7; ++op)
            for (int p : precs)
                for (int64_t np : {(int64_t)0, (int64_t)1, (int64_t)sh[0] * (sh[0] + 1) / 2}) {
                    const size_t b = ri_workspace_bytes(op, sh[0], sh[1], sh[2], np, p);
                    if (op == 7) EXPECT(b == 0);
                    (void)b;
                }
    EXPECT(ri_workspace_bytes(RI_OP_FOCK, 0, 10, 1, 1, RI_FP64) == 0);
    EXPECT(ri_workspace_bytes(RI_OP_FOCK, 10, 10, 1, -1, RI_FP64) == 0);
    for (int p = -1; p <= 4; ++p) (void)ri_packed_b_bytes(1000, 3000, p);
    EXPECT(ri_packed_b_bytes(1000, 3000, RI_FP64) == (size_t)3000 * 136 * 4096 * 8);

    // host buffers standing in for device arrays (never dereferenced by the host layer)
    std::vector<double> dbuf(1 << 16, 0.0);
    std::vector<int32_t> ibuf(1 << 16, 0);
    double* d = dbuf.data();
    int32_t* ip = ibuf.data();
    ri_system s{4, 40, 100, 4, d, d, ip, d, ip, d};
    const int N = 40, na = 100, no = 4;
    const int64_t npairs = 300;

    // argument validation
    int64_t n = 0, bad = 0;
    EXPECT(ri_build_3c(nullptr, 0.0, ip, 0, &n, nullptr, d, 0, nullptr) == RI_E_ARG);
    EXPECT(ri_build_3c(&s, -1.0, ip, 0, &n, nullptr, d, 1 << 20, nullptr) == RI_E_ARG);
    ri_system s0 = s;
    s0.n_occ = 41;
    EXPECT(ri_build_3c(&s0, 0.0, ip, 0, &n, nullptr, d, 1 << 20, nullptr) == RI_E_ARG);
    EXPECT(ri_metric_factor(&s, ip, npairs, d, d, d, d, 9, &bad, d, 1 << 20, nullptr) == RI_E_UNSUPPORTED);
    EXPECT(ri_fock_jk(N, na, no, nullptr, RI_FP64, d, ip, npairs, d, d, d, nullptr, d, 1 << 20, nullptr) == RI_E_ARG);
    EXPECT(ri_fock_jk(N, na, no, d, RI_FP32 | RI_FINAL_FP64, d, ip, npairs, d, d, d, nullptr, d, 1 << 20, nullptr) ==
           RI_E_UNSUPPORTED);
    ri_scf_opts o{10, 6, 1e-10, 1e-8, 0, 0};
    ri_scf_result r;
    ri_scf_opts obad = o;
    obad.diis_n = 9;
    EXPECT(ri_energy(&s, d, RI_FP64, d, ip, npairs, &obad, nullptr, d, d, nullptr, &r, d, 1 << 20, nullptr) ==
           RI_E_ARG);
    obad = o;
    obad.max_purify = -3;
    EXPECT(ri_energy(&s, d, RI_FP64, d, ip, npairs, &obad, nullptr, d, d, nullptr, &r, d, 1 << 20, nullptr) ==
           RI_E_ARG);
    obad = o;
    obad.guess_kind = 7;
    EXPECT(ri_energy(&s, d, RI_FP64, d, ip, npairs, &obad, d, d, d, nullptr, &r, d, 1 << 20, nullptr) ==
           RI_E_UNSUPPORTED);
    EXPECT(ri_energy(&s, d, RI_BF16X3, d, ip, npairs, &o, nullptr, d, d, nullptr, &r, d, 1 << 20, nullptr) ==
           RI_E_UNSUPPORTED);

    // the workspace contract: one byte short of ri_workspace_bytes is refused
    // before any device work, for every operation taking a workspace
    for (int p : {(int)RI_FP64, (int)RI_FP32, (int)RI_BF16X3, (int)RI_BF16X6, RI_FP64 | RI_COMPRESSED}) {
        const size_t b = ri_workspace_bytes(RI_OP_FOCK, N, na, no, npairs, p);
        std::vector<char> ws(b);
        EXPECT(ri_fock_jk(N, na, no, d, p, d, ip, npairs, d, d, d, nullptr, ws.data(), b - 1, nullptr) ==
               RI_E_WORKSPACE);
    }
    for (int p : {(int)RI_FP64, RI_FP32 | RI_FINAL_FP64, RI_BF16X3 | RI_FINAL_FP64, (int)RI_BF16X6}) {
        const size_t b = ri_workspace_bytes(RI_OP_ENERGY, N, na, no, npairs, p);
        std::vector<char> ws(b);
        EXPECT(ri_energy(&s, d, p, d, ip, npairs, &o, nullptr, d, d, nullptr, &r, ws.data(), b - 1, nullptr) ==
               RI_E_WORKSPACE);
    }
    for (int p : {(int)RI_FP64, (int)RI_FP32, (int)RI_BF16X6}) {
        const size_t b = ri_workspace_bytes(RI_OP_GRADIENT, N, na, no, npairs, p);
        std::vector<char> ws(b);
        EXPECT(ri_gradient(&s, ip, npairs, d, p, d, d, d, d, d, ws.data(), b - 1, nullptr) == RI_E_WORKSPACE);
    }
    {
        const size_t b = ri_workspace_bytes(RI_OP_METRIC, N, na, no, npairs, RI_FP64);
        std::vector<char> ws(b);
        EXPECT(ri_metric_factor(&s, ip, npairs, d, d, d, d, RI_FP64, &bad, ws.data(), b - 1, nullptr) ==
               RI_E_WORKSPACE);
    }

    // batched plan: sizes, validation, tuning ranges
    ri_system sys2[3] = {s, s, s};
    sys2[1].n_fn = 130;
    sys2[1].n_aux = 390;
    sys2[1].n_occ = 13;
    sys2[2].n_fn = 600;
    sys2[2].n_aux = 1800;
    sys2[2].n_occ = 60;
    ri_batch_mol mols[3];
    for (auto& m : mols) m = ri_batch_mol{d, d, ip, 200, d, nullptr};
    for (int p : {(int)RI_FP64, (int)RI_FP32, RI_FP32 | RI_FINAL_FP64}) EXPECT(ri_energy_batched_workspace(3, sys2, mols, p) > 0);
    EXPECT(ri_energy_batched_workspace(3, sys2, mols, RI_BF16X3) == 0);
    ri_scf_result res3[3];
    ri_batch_tuning t{};
    t.n_buckets = 5;
    for (int b = 0; b < 5; ++b) { t.gemm_tile[b] = 64; t.syrk_split[b] = 33; }
    EXPECT(ri_energy_batched(3, sys2, mols, RI_FP32, &o, 1, &t, res3, d, 1 << 20, nullptr) == RI_E_ARG);
    {
        const size_t b = ri_energy_batched_workspace(3, sys2, mols, RI_FP64);
        std::vector<char> ws(b);
        EXPECT(ri_energy_batched(3, sys2, mols, RI_FP64, &o, 1, nullptr, res3, ws.data(), b - 1, nullptr) ==
               RI_E_WORKSPACE);
    }

    // a call that reaches the HIP runtime fails there (no device) and reports
    // its text; skipped where a device exists, since these host buffers must
    // never reach a kernel
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
    if (ndev > 0) {
        std::printf("a GPU is present: the RI_E_HIP check is skipped\n");
    } else {
        const size_t b = ri_workspace_bytes(RI_OP_FOCK, N, na, no, npairs, RI_FP64);
        std::vector<char> ws(b);
        EXPECT(ri_fock_jk(N, na, no, d, RI_FP64, d, ip, npairs, d, d, d, nullptr, ws.data(), b, nullptr) == RI_E_HIP);
        EXPECT(std::strlen(ri_last_hip_error()) > 0);
    }

    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("host layer checks passed\n");
    return 0;
}
