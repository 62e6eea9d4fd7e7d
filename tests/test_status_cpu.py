"""Status codes of the C ABI that the host layer decides on its own (no GPU
needed): every code has its own text, a workspace one byte short of
ri_workspace_bytes() is refused before any device work for every operation
that takes one, and on a host without a GPU the first HIP call's failure comes
back as RI_E_HIP with the runtime's text.  The GPU-side outcomes (RI_E_NOT_PD,
RI_E_NO_CONV, RI_E_NO_PURIFY, RI_E_CAPACITY) are in test_gpu_status.py."""
import ctypes

import pytest

import paper_2407_19614_amd as P
from paper_2407_19614_amd import binding as Bd


def test_every_status_has_its_own_text():
    lib = P.lib()
    texts = [lib.ri_status_str(c).decode() for c in range(9)]
    assert len(set(texts)) == 9
    assert lib.ri_status_str(9).decode() == "unknown status"
    assert set(Bd.STATUS) == set(range(9))


def _sys(n_centres, N, na, no, buf):
    a = ctypes.addressof(buf)
    return Bd.RISystem(n_centres, N, na, no, a, a, a, a, a, a)


def test_workspace_one_byte_short_is_refused():
    """ws_bytes = ri_workspace_bytes() - 1 gives RI_E_WORKSPACE; the check
    runs before any HIP call, so this holds without a GPU."""
    lib = P.lib()
    N, na, no, npairs = 40, 100, 4, 300
    buf = ctypes.create_string_buffer(1 << 16)
    s = _sys(4, N, na, no, buf)
    W = lib.ri_workspace_bytes
    n = ctypes.c_int64(0)
    nb = W(Bd.OP_BUILD_3C, N, na, no, 0, P.FP64)
    ws = ctypes.create_string_buffer(nb)
    assert lib.ri_build_3c(ctypes.byref(s), 0.0, buf, 10, ctypes.byref(n), None, ws, nb - 1, None) == 4
    nb = W(Bd.OP_METRIC, N, na, no, npairs, P.FP64)
    ws = ctypes.create_string_buffer(nb)
    bad = ctypes.c_int64(0)
    assert lib.ri_metric_factor(ctypes.byref(s), buf, npairs, buf, buf, buf, buf, P.FP64, ctypes.byref(bad), ws,
                                nb - 1, None) == 4
    assert lib.ri_pack_b(N, na, buf, buf, npairs, buf, P.FP32, ws, nb - 1, None) == 4
    for prec in (P.FP64, P.FP32, P.BF16X3, P.BF16X6, P.FP64 | P.COMPRESSED):
        nb = W(Bd.OP_FOCK, N, na, no, npairs, prec)
        ws = ctypes.create_string_buffer(nb)
        assert lib.ri_fock_jk(N, na, no, buf, prec, buf, buf, npairs, buf, buf, buf, None, ws, nb - 1, None) == 4
    opts = Bd.SCFOpts(10, 6, 1e-10, 1e-8, 0, 0)
    res = Bd.SCFResult()
    for prec in (P.FP64, P.FP32 | P.FINAL_FP64, P.BF16X3 | P.FINAL_FP64):
        nb = W(Bd.OP_ENERGY, N, na, no, npairs, prec)
        ws = ctypes.create_string_buffer(nb)
        assert lib.ri_energy(ctypes.byref(s), buf, prec, buf, buf, npairs, ctypes.byref(opts), None, buf, buf, None,
                             ctypes.byref(res), ws, nb - 1, None) == 4
    for prec in (P.FP64, P.FP32, P.BF16X6):
        nb = W(Bd.OP_GRADIENT, N, na, no, npairs, prec)
        ws = ctypes.create_string_buffer(nb)
        assert lib.ri_gradient(ctypes.byref(s), buf, npairs, buf, prec, buf, buf, buf, buf, buf, ws, nb - 1,
                               None) == 4
    nb = W(Bd.OP_FOCK_DENSITY, N, na, 1, npairs, P.FP64)
    ws = ctypes.create_string_buffer(nb)
    assert lib.ri_fock_jk_density(N, na, buf, buf, npairs, buf, buf, buf, None, ws, nb - 1, None) == 4


def test_purification_limit_is_validated():
    lib = P.lib()
    buf = ctypes.create_string_buffer(1 << 12)
    s = _sys(4, 40, 100, 4, buf)
    opts = Bd.SCFOpts(10, 6, 1e-10, 1e-8, 0, -1)
    res = Bd.SCFResult()
    assert lib.ri_energy(ctypes.byref(s), buf, 0, buf, buf, 10, ctypes.byref(opts), None, buf, buf, None,
                         ctypes.byref(res), buf, 1 << 12, None) == 1


def test_hip_failure_is_reported_without_a_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: the HIP calls succeed")
    lib = P.lib()
    N, na, no, npairs = 40, 100, 4, 100
    nb = lib.ri_workspace_bytes(Bd.OP_FOCK, N, na, no, npairs, P.FP64)
    ws = ctypes.create_string_buffer(nb)
    buf = ctypes.create_string_buffer(1 << 16)
    assert lib.ri_fock_jk(N, na, no, buf, P.FP64, buf, buf, npairs, buf, buf, buf, None, ws, nb, None) == 6
    assert lib.ri_last_hip_error().decode() != ""
