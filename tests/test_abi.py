"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, sizes its workspaces, and rejects bad arguments before any
device call."""
import ctypes
import os
import re

import pytest

import paper_2407_19614_amd as P
from paper_2407_19614_amd import binding as Bd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "ri.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ri_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = P.load_library()
    names = header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(Bd.EXPORTED)


def test_status_strings_and_version():
    assert P.ri_status_str(0) == "ok"
    assert "positive definite" in P.ri_status_str(2)
    assert P.lib().ri_version().startswith(b"libri")


def test_workspace_and_packed_sizes():
    # packed tiles: 16 x 17 / 2 tiles of 64 x 64 per auxiliary function at N=1000
    assert P.packed_b_bytes(1000, 3000, P.FP64) == 3000 * 136 * 4096 * 8
    assert P.packed_b_bytes(1000, 3000, P.FP32) == 3000 * 136 * 4096 * 4
    # split BF16: full square 64 x 64 tiles (16 x 16 per auxiliary), 2 or 3 bf16 parts
    assert P.packed_b_bytes(1000, 3000, P.BF16X3) == 2 * 3000 * 256 * 4096 * 2
    assert P.packed_b_bytes(1000, 3000, P.BF16X6) == 3 * 3000 * 256 * 4096 * 2
    for op in range(4):
        assert P.workspace_bytes(op, 32, 80, 8, 528, P.FP64) > 0
    assert P.workspace_bytes(0, 0, 80, 8, 528, P.FP64) == 0
    assert P.workspace_bytes(2, 32, 80, 8, -1, P.FP64) == 0
    # the compressed form adds the pair map and one slab of packed tiles
    plain = P.workspace_bytes(2, 1000, 3000, 100, 68799, P.FP64)
    comp = P.workspace_bytes(2, 1000, 3000, 100, 68799, P.FP64 | P.COMPRESSED)
    assert comp >= plain + 1000 * 1000 * 4 + 256 * 136 * 4096 * 8
    assert P.workspace_bytes(2, 1000, 3000, 100, 68799, P.BF16X6 | P.COMPRESSED) == 0
    # density Fock build: map, pair weights and two slabs of 8 full N x N matrices
    assert P.workspace_bytes(6, 1000, 3000, 1, 68799, P.FP64) >= 2 * 8 * 1000 * 1000 * 8 + 1000 * 1000 * 4
    # the Fock workspace holds X^T (n_aux * n_occ * Npad doubles)
    assert P.workspace_bytes(2, 1000, 3000, 100, 68799, P.FP64) >= 3000 * 100 * 1024 * 8


def test_bad_arguments_rejected_before_device_work():
    lib = P.lib()
    n = ctypes.c_int64(0)
    assert lib.ri_build_3c(None, 0.0, None, 0, ctypes.byref(n), None, None, 0, None) == 1
    s = Bd.RISystem(0, 0, 0, 0, None, None, None, None, None, None)
    assert lib.ri_build_3c(ctypes.byref(s), 0.0, None, 0, ctypes.byref(n), None, None, 0, None) == 1
    assert lib.ri_fock_jk(0, 10, 2, None, 0, None, None, 0, None, None, None, None, None, 0, None) == 1
    assert lib.ri_fock_jk(10, 10, 20, None, 0, None, None, 0, None, None, None, None, None, 0, None) == 1
    # B may be NULL only with the compressed flag; the flag needs FP64 or FP32
    ws = ctypes.create_string_buffer(64)
    # split BF16 keeps n_occ <= 128 (eight 16-column MFMA tiles)
    assert lib.ri_fock_jk(200, 10, 129, ws, P.BF16X6, None, None, 0, ws, ws, ws, None, ws, 64, None) == 7
    assert lib.ri_fock_jk(10, 10, 2, None, 0, None, None, 0, ws, ws, ws, None, ws, 64, None) == 1
    assert lib.ri_fock_jk(10, 10, 2, None, P.BF16X6 | P.COMPRESSED, None, None, 0, ws, ws, ws, None, ws, 64,
                          None) not in (0, 1)
    bad = ctypes.c_int64(0)
    assert lib.ri_metric_factor(ctypes.byref(s), None, 0, None, None, None, None, 0, ctypes.byref(bad), None, 0,
                                None) == 1
    opts = Bd.SCFOpts(0, 6, 1e-10, 1e-8, 0)
    res = Bd.SCFResult()
    assert lib.ri_energy(ctypes.byref(s), None, 0, None, None, 0, ctypes.byref(opts), None, None, None, None,
                         ctypes.byref(res), None, 0, None) == 1
    # batched: an out-of-range launch shape is rejected before anything else is read
    sysarr = (Bd.RISystem * 1)(s)
    mols = (Bd.BatchMol * 1)()
    ws = ctypes.create_string_buffer(256)
    opts6 = Bd.SCFOpts(10, 6, 1e-10, 1e-8, 0)
    res1 = (Bd.SCFResult * 1)()
    for tile, split, nb in ((96, 2, 1), (64, 0, 1), (128, 17, 1), (64, 2, 0), (64, 2, 9)):
        t = Bd.BatchTuning()
        t.n_buckets = nb
        for b in range(Bd.TUNE_BUCKETS):
            t.gemm_tile[b], t.syrk_split[b] = tile, split
        assert lib.ri_energy_batched(1, ctypes.byref(sysarr), ctypes.byref(mols), 0, ctypes.byref(opts6), 0,
                                     ctypes.byref(t), ctypes.byref(res1), ws, 256, None) == 1
    assert lib.ri_batch_autotune(1, ctypes.byref(sysarr), ctypes.byref(mols), 0, None, ws, 256, None) == 1
    assert ctypes.sizeof(Bd.BatchTuning) == 4 + 4 * 8 * 4
    # the final-FP64 flag goes with FP32 exchange only
    assert lib.ri_energy_batched(1, ctypes.byref(sysarr), ctypes.byref(mols), P.FP64 | P.FINAL_FP64,
                                 ctypes.byref(opts6), 0, None, ctypes.byref(res1), ws, 256, None) == 7
    assert lib.ri_energy_batched(1, ctypes.byref(sysarr), ctypes.byref(mols), P.FP32 | P.FINAL_FP64,
                                 ctypes.byref(opts6), 0, None, ctypes.byref(res1), ws, 256, None) == 1
    assert lib.ri_energy_batched_workspace(1, ctypes.byref(sysarr), ctypes.byref(mols),
                                           P.BF16X3 | P.FINAL_FP64) == 0
    assert ctypes.sizeof(Bd.BatchMol) == 6 * 8
    # the final-FP64 flag: ri_energy (and its workspace) with resident FP32 or split-BF16 B only
    W = lib.ri_workspace_bytes
    assert W(3, 100, 300, 10, 1000, P.FP32 | P.FINAL_FP64) > W(3, 100, 300, 10, 1000, P.FP32) > 0
    assert W(3, 100, 300, 10, 1000, P.FP32 | P.FINAL_FP64) == W(3, 100, 300, 10, 1000, P.FP64)
    for prec in (P.BF16X3, P.BF16X6):
        # the split-BF16 final build adds FP64 X^T and one slab of unpacked FP64 tiles
        assert W(3, 100, 300, 10, 1000, prec | P.FINAL_FP64) > W(3, 100, 300, 10, 1000, prec) > 0
        # their gradient reads B_c slab by slab, as the compressed FP64 form does
        assert W(4, 100, 300, 10, 1000, prec) == W(4, 100, 300, 10, 1000, P.FP64 | P.COMPRESSED)
    for prec in (P.FP64 | P.FINAL_FP64, P.FP32 | P.COMPRESSED | P.FINAL_FP64, P.BF16X6 | P.COMPRESSED):
        assert W(3, 100, 300, 10, 1000, prec) == 0
    assert W(2, 100, 300, 10, 1000, P.FP32 | P.FINAL_FP64) == 0      # Fock build
    assert W(4, 100, 300, 10, 1000, P.FP32 | P.FINAL_FP64) == 0      # gradient
    assert lib.ri_fock_jk(10, 10, 2, ws, P.FP32 | P.FINAL_FP64, None, None, 0, ws, ws, ws, None, ws, 64,
                          None) == 7
    # ri_pack_b: sizes and pointers first, then the precision (no flags)
    assert lib.ri_pack_b(0, 10, ws, ws, 1, ws, P.FP64, ws, 256, None) == 1
    assert lib.ri_pack_b(10, 10, None, ws, 1, ws, P.FP64, ws, 256, None) == 1
    assert lib.ri_pack_b(10, 10, ws, ws, 1, None, P.FP64, ws, 256, None) == 1
    assert lib.ri_pack_b(10, 10, ws, ws, 1, ws, P.FP64 | P.COMPRESSED, ws, 256, None) == 7
    assert lib.ri_pack_b(10, 10, ws, ws, 1, ws, 9, ws, 256, None) == 7


def test_product_path_has_no_oracle_import():
    pkg = os.path.join(ROOT, "paper_2407_19614_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
