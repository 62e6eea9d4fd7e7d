"""ctypes binding of libri's C ABI (include/ri.h) with torch device buffers.

Argument marshalling only: sizes, pointers and the current HIP stream go to
the library; no arithmetic of the method happens here.  There is no CPU
fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_void_p, c_char_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libri.so")

FP64, FP32, BF16X3, BF16X6 = 0, 1, 2, 3
COMPRESSED = 0x10          # flag: B not resident, decompressed per auxiliary slab each call
COMPRESSED_SLAB = 256
FINAL_FP64 = 0x20          # SCF flag (FP32, BF16X3, BF16X6): one FP64 exchange build after the SCF
OP_BUILD_3C, OP_METRIC, OP_FOCK, OP_ENERGY, OP_GRADIENT = range(5)
OP_FOCK_DENSITY = 6
STATUS = {0: "RI_OK", 1: "RI_E_ARG", 2: "RI_E_NOT_PD", 3: "RI_E_NO_CONV", 4: "RI_E_WORKSPACE",
          5: "RI_E_CAPACITY", 6: "RI_E_HIP", 7: "RI_E_UNSUPPORTED", 8: "RI_E_NO_PURIFY"}


class RIError(RuntimeError):
    def __init__(self, code, where, extra=""):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} ({ri_status_str(code)}){extra}")


class RISystem(ctypes.Structure):
    _fields_ = [("n_centres", c_int32), ("n_fn", c_int32), ("n_aux", c_int32), ("n_occ", c_int32),
                ("xyz", c_void_p), ("Z", c_void_p), ("fn_centre", c_void_p), ("fn_exp", c_void_p),
                ("aux_centre", c_void_p), ("aux_exp", c_void_p)]


class SCFOpts(ctypes.Structure):
    _fields_ = [("max_iter", c_int32), ("diis_n", c_int32), ("tol_E", c_double), ("tol_err", c_double),
                ("guess_kind", c_int32), ("max_purify", c_int32)]


class SCFResult(ctypes.Structure):
    _fields_ = [("E_total", c_double), ("E_nuc", c_double), ("E_1e", c_double), ("E_J", c_double),
                ("E_K", c_double), ("n_iter", c_int32), ("converged", c_int32), ("last_dE", c_double),
                ("max_err", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RIMlp(ctypes.Structure):
    _fields_ = [("params", c_void_p), ("mu", c_void_p), ("sigma", c_void_p)]


NFEAT, WIDTH = 8, 256
OFF_W1 = 0
OFF_B1 = OFF_W1 + NFEAT * WIDTH
OFF_W2 = OFF_B1 + WIDTH
OFF_B2 = OFF_W2 + WIDTH * WIDTH
OFF_W3 = OFF_B2 + WIDTH
OFF_B3 = OFF_W3 + WIDTH
NPARAM = OFF_B3 + 1
MLP_FP32, MLP_BF16 = 0, 1
OP_MLP = 5

class BatchMol(ctypes.Structure):
    _fields_ = [("B", c_void_p), ("Bc", c_void_p), ("pairs", c_void_p), ("n_pairs", c_int64),
                ("C_occ", c_void_p), ("F", c_void_p)]


TUNE_BUCKETS = 8


class BatchTuning(ctypes.Structure):
    """Launch shapes of the batched SCF per size bucket (bucket b: N in
    (128 b, 128 (b + 1)]); see ri_batch_autotune."""
    _fields_ = [("n_buckets", c_int32), ("gemm_tile", c_int32 * TUNE_BUCKETS),
                ("syrk_split", c_int32 * TUNE_BUCKETS), ("gemm_ms", ctypes.c_float * TUNE_BUCKETS),
                ("syrk_ms", ctypes.c_float * TUNE_BUCKETS)]

    def as_dict(self):
        n = self.n_buckets
        return {"n_buckets": n, "gemm_tile": list(self.gemm_tile[:n]), "syrk_split": list(self.syrk_split[:n]),
                "gemm_ms": [round(x, 4) for x in self.gemm_ms[:n]], "syrk_ms": [round(x, 4) for x in self.syrk_ms[:n]]}


_LIB = None
_SIGS = {
    "ri_version": (c_char_p, []),
    "ri_status_str": (c_char_p, [c_int32]),
    "ri_last_hip_error": (c_char_p, []),
    "ri_packed_b_bytes": (c_size_t, [c_int32, c_int32, c_int32]),
    "ri_workspace_bytes": (c_size_t, [c_int32, c_int32, c_int32, c_int32, c_int64, c_int32]),
    "ri_build_3c": (c_int32, [POINTER(RISystem), c_double, c_void_p, c_int64, POINTER(c_int64), c_void_p,
                              c_void_p, c_size_t, c_void_p]),
    "ri_metric_factor": (c_int32, [POINTER(RISystem), c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_int32, POINTER(c_int64), c_void_p, c_size_t, c_void_p]),
    "ri_fock_jk": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_int64, c_void_p,
                             c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "ri_fock_jk_noalloc": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_int64,
                                     c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ri_fock_jk_timed": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_int64,
                                   c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p,
                                   ctypes.POINTER(c_void_p)]),
    "ri_energy": (c_int32, [POINTER(RISystem), c_void_p, c_int32, c_void_p, c_void_p, c_int64, POINTER(SCFOpts),
                            c_void_p, c_void_p, c_void_p, c_void_p, POINTER(SCFResult), c_void_p, c_size_t,
                            c_void_p]),
    "ri_pair_features": (c_int32, [POINTER(RISystem), c_void_p, c_int64, c_void_p, c_void_p]),
    "ri_mlp_forward": (c_int32, [POINTER(RIMlp), c_void_p, c_int64, c_void_p, c_int32, c_void_p, c_size_t, c_void_p]),
    "ri_mlp_train_step": (c_int32, [POINTER(RIMlp), c_void_p, c_void_p, c_int32, ctypes.c_float, c_void_p, c_void_p,
                                    c_int64, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "ri_density_to_pairs": (c_int32, [c_int32, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "ri_density_from_pairs": (c_int32, [c_int32, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "ri_pair_delta_features": (c_int32, [POINTER(RISystem), c_void_p, c_void_p, c_int64, c_void_p, c_void_p,
                                         c_void_p]),
    "ri_density_change_pairs": (c_int32, [c_int32, c_void_p, c_int64, c_void_p, c_void_p, ctypes.c_float, c_void_p,
                                          c_void_p]),
    "ri_density_add_pairs": (c_int32, [c_int32, c_void_p, c_int64, c_void_p, c_double, c_void_p, c_void_p,
                                       c_void_p]),
    "ri_energy_batched_workspace": (c_size_t, [c_int32, c_void_p, c_void_p, c_int32]),
    "ri_batch_autotune": (c_int32, [c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p]),
    "ri_energy_batched": (c_int32, [c_int32, c_void_p, c_void_p, c_int32, POINTER(SCFOpts), c_int32, c_void_p,
                                    c_void_p, c_void_p, c_size_t, c_void_p]),
    "ri_fock_jk_density": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_size_t, c_void_p]),
    "ri_md_verlet": (c_int32, [c_int32, c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p]),
    "ri_md_kinetic": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ri_pack_b": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_int64, c_void_p, c_int32, c_void_p, c_size_t,
                            c_void_p]),
    "ri_gradient": (c_int32, [POINTER(RISystem), c_void_p, c_int64, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                              c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
}
EXPORTED = tuple(_SIGS)


def load_library(path: str = LIB_PATH):
    """Load libri.so once; raise if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2407_19614_amd.build`")
        lib_ = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib_, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib_
    return _LIB


def lib():
    return load_library()


def ri_status_str(code: int) -> str:
    return lib().ri_status_str(int(code)).decode()


def workspace_bytes(op, N, n_aux, n_occ, n_pairs, prec=FP64) -> int:
    return int(lib().ri_workspace_bytes(op, N, n_aux, n_occ, n_pairs, prec))


def packed_b_bytes(N, n_aux, prec=FP64) -> int:
    return int(lib().ri_packed_b_bytes(N, n_aux, prec))


def _check(code, where):
    if code != 0:
        extra = ""
        if code == 6:
            extra = ": " + lib().ri_last_hip_error().decode()
        raise RIError(code, where, extra)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class RIProblem:
    """Device-resident state of one molecular system.

    Holds the system arrays, pair list, fitted tensors and workspace as torch
    tensors on the current HIP device, and calls the five entry points.
    """

    def __init__(self, system, device="cuda", prec=FP64, compressed=False):
        import torch
        self.torch = torch
        self.system = system
        self.device = torch.device(device)
        self.prec = prec
        self.compressed = bool(compressed)
        dev = self.device
        f64 = dict(dtype=torch.float64, device=dev)
        i32 = dict(dtype=torch.int32, device=dev)
        self.xyz = torch.tensor(np.ascontiguousarray(system.xyz), **f64)
        self.Z = torch.tensor(np.ascontiguousarray(system.Z), **f64)
        self.fn_centre = torch.tensor(np.ascontiguousarray(system.fn_centre, dtype=np.int32), **i32)
        self.fn_exp = torch.tensor(np.ascontiguousarray(system.fn_exp), **f64)
        self.aux_centre = torch.tensor(np.ascontiguousarray(system.aux_centre, dtype=np.int32), **i32)
        self.aux_exp = torch.tensor(np.ascontiguousarray(system.aux_exp), **f64)
        self.N, self.n_aux, self.n_occ = system.N, system.n_aux, system.n_occ
        self.c_sys = RISystem(system.n_centres, self.N, self.n_aux, self.n_occ,
                              self.xyz.data_ptr(), self.Z.data_ptr(), self.fn_centre.data_ptr(),
                              self.fn_exp.data_ptr(), self.aux_centre.data_ptr(), self.aux_exp.data_ptr())
        self._ws = None
        self.pairs = self.T = self.L = self.Linv = self.B = None
        self.n_pairs = None

    # -- helpers
    def stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def workspace(self, nbytes):
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = self.torch.empty(max(int(nbytes), 256), dtype=self.torch.uint8, device=self.device)
        return self._ws

    @property
    def pflag(self):
        """The precision argument of the calls that take B (with the compressed flag)."""
        return self.prec | (COMPRESSED if self.compressed else 0)

    def _ws_for(self, op, prec=None):
        prec = self.prec if prec is None else prec
        if self.compressed and op in (OP_FOCK, OP_ENERGY, OP_GRADIENT):
            prec |= COMPRESSED
        nb = workspace_bytes(op, self.N, self.n_aux, self.n_occ, max(self.n_pairs or 0, 0), prec)
        if nb == 0:
            raise RIError(1, "ri_workspace_bytes")
        return self.workspace(nb), nb

    # -- entry points
    def build_3c(self, tau=None):
        torch = self.torch
        tau = self.system.tau if tau is None else tau
        ws = self.workspace(workspace_bytes(OP_BUILD_3C, self.N, self.n_aux, self.n_occ, 0, FP64))
        n = c_int64(0)
        dummy = torch.empty(2, dtype=torch.int32, device=self.device)
        code = lib().ri_build_3c(ctypes.byref(self.c_sys), float(tau), _ptr(dummy), 0, ctypes.byref(n), None,
                                 _ptr(ws), ws.numel(), self.stream())
        if code not in (0, 5):
            _check(code, "ri_build_3c")
        self.n_pairs = int(n.value)
        self.pairs = torch.empty((max(self.n_pairs, 1), 2), dtype=torch.int32, device=self.device)
        self.T = torch.empty((self.n_aux, max(self.n_pairs, 1)), dtype=torch.float64, device=self.device)
        code = lib().ri_build_3c(ctypes.byref(self.c_sys), float(tau), _ptr(self.pairs), self.pairs.shape[0],
                                 ctypes.byref(n), _ptr(self.T), _ptr(ws), ws.numel(), self.stream())
        _check(code, "ri_build_3c")
        return self.n_pairs

    def metric_factor(self, prec=None, pack=True):
        torch = self.torch
        prec = self.prec if prec is None else prec
        self.prec = prec
        self.L = torch.empty((self.n_aux, self.n_aux), dtype=torch.float64, device=self.device)
        self.Linv = torch.empty_like(self.L)
        self.B = None
        if pack and not self.compressed:
            self.B = torch.empty(packed_b_bytes(self.N, self.n_aux, prec), dtype=torch.uint8, device=self.device)
        ws, nb = self._ws_for(OP_METRIC, prec)
        bad = c_int64(-1)
        code = lib().ri_metric_factor(ctypes.byref(self.c_sys), _ptr(self.pairs), self.n_pairs, _ptr(self.T),
                                      _ptr(self.L), _ptr(self.Linv), _ptr(self.B), prec, ctypes.byref(bad),
                                      _ptr(ws), nb, self.stream())
        _check(code, "ri_metric_factor", ) if code != 2 else None
        if code == 2:
            raise RIError(code, "ri_metric_factor", f": pivot {bad.value}")
        return self

    def pack_b(self, prec):
        """The packed B of this problem (after metric_factor) in another
        precision, from the fitted tensor: a new device tensor."""
        B = self.torch.empty(packed_b_bytes(self.N, self.n_aux, prec), dtype=self.torch.uint8, device=self.device)
        ws, nb = self._ws_for(OP_METRIC, prec)
        _check(lib().ri_pack_b(self.N, self.n_aux, _ptr(self.T), _ptr(self.pairs), self.n_pairs, _ptr(B), prec,
                               _ptr(ws), nb, self.stream()), "ri_pack_b")
        return B

    @property
    def Bc(self):
        return self.T

    def fock_jk(self, C_occ, J=None, K=None, gamma=None):
        torch = self.torch
        C_occ = C_occ.contiguous()
        J = torch.empty((self.N, self.N), dtype=torch.float64, device=self.device) if J is None else J
        K = torch.empty_like(J) if K is None else K
        gamma = torch.empty(self.n_aux, dtype=torch.float64, device=self.device) if gamma is None else gamma
        ws, nb = self._ws_for(OP_FOCK)
        code = lib().ri_fock_jk(self.N, self.n_aux, self.n_occ, _ptr(self.B), self.pflag, _ptr(self.T),
                                _ptr(self.pairs), self.n_pairs, _ptr(C_occ), _ptr(J), _ptr(K), _ptr(gamma),
                                _ptr(ws), nb, self.stream())
        _check(code, "ri_fock_jk")
        return J, K, gamma

    def fock_jk_noalloc(self, C_occ, J, K, gamma=None):
        """ri_fock_jk_noalloc into caller-owned J, K (and gamma): the library's
        static scratch instead of a workspace.  Returns the status code."""
        C_occ = C_occ.contiguous()
        return lib().ri_fock_jk_noalloc(self.N, self.n_aux, self.n_occ, _ptr(self.B), self.pflag, _ptr(self.T),
                                        _ptr(self.pairs), self.n_pairs, _ptr(C_occ), _ptr(J), _ptr(K), _ptr(gamma),
                                        self.stream())

    def fock_jk_timed(self, C_occ, J, K, gamma, events):
        """ri_fock_jk with four torch.cuda.Event objects recorded by the
        library: start, end of gamma/J (side stream), end of X, end.  Phases:
        gamma/J = e0..e1 (e2..e1 for the split-BF16 forms, whose gamma/J
        starts after X), X = e0..e2, SYRK = e2..e3 (see fock_phases)."""
        C_occ = C_occ.contiguous()
        ws, nb = self._ws_for(OP_FOCK)
        arr = (c_void_p * 4)(*[ctypes.c_void_p(e.cuda_event) for e in events])
        code = lib().ri_fock_jk_timed(self.N, self.n_aux, self.n_occ, _ptr(self.B), self.pflag, _ptr(self.T),
                                      _ptr(self.pairs), self.n_pairs, _ptr(C_occ), _ptr(J), _ptr(K), _ptr(gamma),
                                      _ptr(ws), nb, self.stream(), arr)
        _check(code, "ri_fock_jk_timed")

    @staticmethod
    def fock_phases(events, bf16=False):
        """(gamma/J, X, SYRK) in ms from the events of one fock_jk_timed call
        (bf16: a split-BF16 build, whose gamma/J runs beside the SYRK)."""
        e0, e1, e2, e3 = events
        return (e2 if bf16 else e0).elapsed_time(e1), e0.elapsed_time(e2), e2.elapsed_time(e3)

    def pair_features(self):
        torch = self.torch
        f = torch.empty((max(self.n_pairs, 1), NFEAT), dtype=torch.float32, device=self.device)
        _check(lib().ri_pair_features(ctypes.byref(self.c_sys), _ptr(self.pairs), self.n_pairs, _ptr(f),
                                      self.stream()), "ri_pair_features")
        return f[: self.n_pairs]

    def density_to_pairs(self, D):
        torch = self.torch
        d = torch.empty(max(self.n_pairs, 1), dtype=torch.float32, device=self.device)
        _check(lib().ri_density_to_pairs(self.N, _ptr(self.pairs), self.n_pairs, _ptr(D.contiguous()), _ptr(d),
                                         self.stream()), "ri_density_to_pairs")
        return d[: self.n_pairs]

    def pair_delta_features(self, xyz_prev, D_prev):
        """Features of this problem's pairs for the density change from the
        previous geometry (positions xyz_prev, converged density D_prev)."""
        torch = self.torch
        f = torch.empty((max(self.n_pairs, 1), NFEAT), dtype=torch.float32, device=self.device)
        _check(lib().ri_pair_delta_features(ctypes.byref(self.c_sys), _ptr(xyz_prev.contiguous()), _ptr(self.pairs),
                                            self.n_pairs, _ptr(D_prev.contiguous()), _ptr(f), self.stream()),
               "ri_pair_delta_features")
        return f[: self.n_pairs]

    def density_change_pairs(self, D_new, D_prev, scale):
        torch = self.torch
        d = torch.empty(max(self.n_pairs, 1), dtype=torch.float32, device=self.device)
        _check(lib().ri_density_change_pairs(self.N, _ptr(self.pairs), self.n_pairs, _ptr(D_new.contiguous()),
                                             _ptr(D_prev.contiguous()), float(scale), _ptr(d), self.stream()),
               "ri_density_change_pairs")
        return d[: self.n_pairs]

    def density_add_pairs(self, d, scale, D_prev):
        torch = self.torch
        D = torch.empty((self.N, self.N), dtype=torch.float64, device=self.device)
        _check(lib().ri_density_add_pairs(self.N, _ptr(self.pairs), self.n_pairs, _ptr(d.contiguous()), float(scale),
                                          _ptr(D_prev.contiguous()), _ptr(D), self.stream()), "ri_density_add_pairs")
        return D

    def density_from_pairs(self, d):
        torch = self.torch
        D = torch.empty((self.N, self.N), dtype=torch.float64, device=self.device)
        _check(lib().ri_density_from_pairs(self.N, _ptr(self.pairs), self.n_pairs, _ptr(d.contiguous()), _ptr(D),
                                           self.stream()), "ri_density_from_pairs")
        return D

    def fock_jk_density(self, D, J=None, K=None, gamma=None):
        """J and K of a density matrix given without orbitals."""
        torch = self.torch
        D = D.contiguous()
        J = torch.empty((self.N, self.N), dtype=torch.float64, device=self.device) if J is None else J
        K = torch.empty_like(J) if K is None else K
        nb = workspace_bytes(OP_FOCK_DENSITY, self.N, self.n_aux, 1, self.n_pairs, FP64)
        ws = self.workspace(nb)
        code = lib().ri_fock_jk_density(self.N, self.n_aux, _ptr(self.T), _ptr(self.pairs), self.n_pairs, _ptr(D),
                                        _ptr(J), _ptr(K), _ptr(gamma), _ptr(ws), nb, self.stream())
        _check(code, "ri_fock_jk_density")
        return J, K

    def energy(self, max_iter=100, diis_n=6, tol_E=1e-10, tol_err=1e-8, guess=None, raise_on_noconv=True,
               guess_density=None, density_fock=False, final_fp64=False, max_purify=0):
        """SCF.  guess: C_occ start; guess_density: density start, through its
        natural orbitals, or (density_fock=True) through the occupied space of
        its own Fock matrix (J and K built from the density).  final_fp64
        (FP32 and split-BF16 problems): one FP64 exchange build at the
        converged density gives the reported energy (RI_FINAL_FP64)."""
        torch = self.torch
        kind = 0 if guess is None else 1
        if guess_density is not None:
            kind, guess = (3 if density_fock else 2), guess_density
        opts = SCFOpts(max_iter, diis_n, tol_E, tol_err, kind, max_purify)
        C = torch.empty((self.N, self.n_occ), dtype=torch.float64, device=self.device)
        F = torch.empty((self.N, self.N), dtype=torch.float64, device=self.device)
        D = torch.empty_like(F)
        res = SCFResult()
        fin = FINAL_FP64 if final_fp64 else 0
        ws, nb = self._ws_for(OP_ENERGY, self.prec | fin)
        g = None if guess is None else guess.contiguous()
        code = lib().ri_energy(ctypes.byref(self.c_sys), _ptr(self.B), self.pflag | fin, _ptr(self.T), _ptr(self.pairs),
                               self.n_pairs, ctypes.byref(opts), _ptr(g), _ptr(C), _ptr(F), _ptr(D),
                               ctypes.byref(res), _ptr(ws), nb, self.stream())
        if code == 3 and not raise_on_noconv:
            return res.as_dict(), C, F, D
        _check(code, "ri_energy")
        self.C_occ, self.F, self.D = C, F, D
        return res.as_dict(), C, F, D

    def record_stream(self, stream):
        """Marks every device tensor of this problem as used on `stream`, so the
        caching allocator does not reuse its memory on the stream it was
        allocated on while work queued on `stream` may still read it."""
        for name in ("xyz", "Z", "fn_centre", "fn_exp", "aux_centre", "aux_exp", "pairs", "T", "L", "Linv", "B",
                     "_ws"):
            t = getattr(self, name, None)
            if t is not None:
                t.record_stream(stream)

    def gradient(self, C_occ=None, F=None):
        torch = self.torch
        C_occ = self.C_occ if C_occ is None else C_occ
        F = self.F if F is None else F
        g = torch.empty((self.system.n_centres, 3), dtype=torch.float64, device=self.device)
        ws, nb = self._ws_for(OP_GRADIENT)
        code = lib().ri_gradient(ctypes.byref(self.c_sys), _ptr(self.pairs), self.n_pairs, _ptr(self.B), self.pflag,
                                 _ptr(self.T), _ptr(self.Linv), _ptr(C_occ), _ptr(F), _ptr(g), _ptr(ws), nb,
                                 self.stream())
        _check(code, "ri_gradient")
        return g


class MLP:
    """Device parameters of the learned-start network plus Adam moments."""

    def __init__(self, params, mu, sigma, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.params = torch.tensor(np.asarray(params, dtype=np.float32), device=self.device)
        assert self.params.numel() == NPARAM
        self.mu = torch.tensor(np.asarray(mu, dtype=np.float32), device=self.device)
        self.sigma = torch.tensor(np.asarray(sigma, dtype=np.float32), device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.c = RIMlp(self.params.data_ptr(), self.mu.data_ptr(), self.sigma.data_ptr())
        self._ws = None

    def _ws_for(self, n):
        nb = workspace_bytes(OP_MLP, 1, 1, 1, int(n), FP64)
        if self._ws is None or self._ws.numel() < nb:
            self._ws = self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)
        return self._ws, nb

    def stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def forward(self, feat, prec=MLP_FP32):
        n = feat.shape[0]
        y = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        ws, nb = self._ws_for(n)
        _check(lib().ri_mlp_forward(ctypes.byref(self.c), _ptr(feat.contiguous()), n, _ptr(y), prec, _ptr(ws), nb,
                                    self.stream()), "ri_mlp_forward")
        return y

    def train_step(self, feat, target, lr, want_grad=False):
        n = feat.shape[0]
        self.step += 1
        loss = self.torch.empty(1, dtype=self.torch.float32, device=self.device)
        g = self.torch.empty_like(self.params) if want_grad else None
        ws, nb = self._ws_for(n)
        _check(lib().ri_mlp_train_step(ctypes.byref(self.c), _ptr(self.m), _ptr(self.v), self.step, float(lr),
                                       _ptr(feat.contiguous()), _ptr(target.contiguous()), n, _ptr(loss), _ptr(g),
                                       _ptr(ws), nb, self.stream()), "ri_mlp_train_step")
        return (loss, g) if want_grad else loss


def pack_params(p):
    """Flat parameter vector (layout of include/ri.h) from a dict of arrays."""
    return np.concatenate([np.asarray(p["W1"]).reshape(-1), p["b1"], np.asarray(p["W2"]).reshape(-1), p["b2"],
                           p["w3"], p["b3"]]).astype(np.float32)


def unpack_params(v):
    v = np.asarray(v, dtype=np.float64)
    return {"W1": v[OFF_W1:OFF_B1].reshape(NFEAT, WIDTH), "b1": v[OFF_B1:OFF_W2],
            "W2": v[OFF_W2:OFF_B2].reshape(WIDTH, WIDTH), "b2": v[OFF_B2:OFF_W3],
            "w3": v[OFF_W3:OFF_B3], "b3": v[OFF_B3:OFF_B3 + 1]}


def _batch_args(problems, want_fock=False):
    import torch
    n = len(problems)
    dev = problems[0].device
    sysarr = (RISystem * n)(*[p.c_sys for p in problems])
    Cs = [torch.empty((p.N, p.n_occ), dtype=torch.float64, device=dev) for p in problems]
    Fs = [torch.empty((p.N, p.N), dtype=torch.float64, device=dev) for p in problems] if want_fock else [None] * n
    mols = (BatchMol * n)(*[BatchMol(p.B.data_ptr(), p.T.data_ptr(), p.pairs.data_ptr(), p.n_pairs,
                                     Cs[i].data_ptr(), None if Fs[i] is None else Fs[i].data_ptr())
                            for i, p in enumerate(problems)])
    return n, dev, sysarr, mols, Cs, Fs


def _batch_ws(n, sysarr, mols, prec, dev):
    import torch
    nb = int(lib().ri_energy_batched_workspace(n, ctypes.byref(sysarr), ctypes.byref(mols), prec))
    if nb == 0:
        raise RIError(7, "ri_energy_batched_workspace")
    return torch.empty(nb, dtype=torch.uint8, device=dev), nb


def batch_workspace_bytes(problems, prec=FP64):
    """Workspace bytes energy_batched allocates for these problems."""
    n, _, sysarr, mols, _, _ = _batch_args(problems)
    return int(lib().ri_energy_batched_workspace(n, ctypes.byref(sysarr), ctypes.byref(mols), prec))


_PREP_STREAMS = {}


def prepare_batch(systems, prec=FP64, workers=4, device="cuda"):
    """RIProblem objects for independent systems, each after build_3c and
    metric_factor in `prec` (the FINAL_FP64 flag is ignored here: its batched
    SCF needs the FP32 B only).  The setups of different systems share no data,
    and each is a chain of small launches with host reads of sizes, so
    `workers` host threads each issue their share on a stream of their own
    and the launches of several systems overlap on the device.  The streams
    are made once per device and reused, so memory freed by one batch is
    found again by the next (the caching allocator keeps freed blocks per
    stream).  Returns when every system's data is complete on the device."""
    import threading
    import torch
    dev = torch.device(device)
    key = (dev.index if dev.index is not None else torch.cuda.current_device(), int(workers))
    if key not in _PREP_STREAMS:
        _PREP_STREAMS[key] = [torch.cuda.Stream(device=dev) for _ in range(workers)]
    streams = _PREP_STREAMS[key]
    out = [None] * len(systems)
    errors = []

    def work(k):
        try:
            with torch.cuda.stream(streams[k]):
                for i in range(k, len(systems), workers):
                    base = prec & ~FINAL_FP64
                    pr = RIProblem(systems[i], device=dev, prec=base)
                    pr.build_3c()
                    pr.metric_factor(base)
                    out[i] = pr
        except BaseException as e:        # re-raised on the calling thread
            errors.append(e)
        finally:
            streams[k].synchronize()

    threads = [threading.Thread(target=work, args=(k,)) for k in range(workers)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    if errors:
        raise errors[0]
    cur = torch.cuda.current_stream(dev)
    for pr in out:
        pr.record_stream(cur)   # allocated on a worker stream, used on the caller's
    return out


class PreparedBatch:
    """prepare_batch running on a host thread of its own (its launches go to
    the worker streams, so they overlap whatever the caller's stream runs,
    e.g. the SCF of the previous batch).  result() waits for it and returns
    the problems, recorded for use on the calling thread's current stream."""

    def __init__(self, systems, prec=FP64, workers=4, device="cuda"):
        import threading
        self._out, self._err = None, None

        def run():
            try:
                self._out = prepare_batch(systems, prec, workers, device)
            except BaseException as e:     # re-raised by result()
                self._err = e
        self._thread = threading.Thread(target=run)
        self._thread.start()

    def result(self):
        import torch
        self._thread.join()
        if self._err is not None:
            raise self._err
        cur = torch.cuda.current_stream()
        for pr in self._out:
            pr.record_stream(cur)
        return self._out


def batch_autotune(problems, prec=FP64):
    """Times the candidate launch shapes of the batched SCF on these problems
    (each after build_3c and metric_factor in `prec`) and returns the chosen
    BatchTuning (pass it to energy_batched)."""
    import torch
    n, dev, sysarr, mols, _, _ = _batch_args(problems)
    ws, nb = _batch_ws(n, sysarr, mols, prec, dev)
    out = BatchTuning()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    code = lib().ri_batch_autotune(n, ctypes.byref(sysarr), ctypes.byref(mols), prec, ctypes.byref(out), _ptr(ws),
                                   nb, stream)
    _check(code, "ri_batch_autotune")
    del ws
    return out


def energy_batched(problems, prec=FP64, max_iter=100, diis_n=6, tol_E=1e-10, tol_err=1e-8, use_graph=True,
                   want_fock=False, raise_on_noconv=True, tuning=None, max_purify=0):
    """Lockstep SCF for a list of RIProblem objects (each after build_3c and
    metric_factor in precision `prec`), with launch shapes from `tuning`
    (a BatchTuning, or None for the defaults).  Returns (results, C_occ
    list, F list)."""
    import torch
    n, dev, sysarr, mols, Cs, Fs = _batch_args(problems, want_fock)
    ws, nb = _batch_ws(n, sysarr, mols, prec, dev)
    res = (SCFResult * n)()
    opts = SCFOpts(max_iter, diis_n, tol_E, tol_err, 0, max_purify)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    code = lib().ri_energy_batched(n, ctypes.byref(sysarr), ctypes.byref(mols), prec, ctypes.byref(opts),
                                   1 if use_graph else 0, None if tuning is None else ctypes.byref(tuning),
                                   ctypes.byref(res), _ptr(ws), nb, stream)
    if code not in (0, 3, 8) or (code in (3, 8) and raise_on_noconv):
        _check(code, "ri_energy_batched")
    del ws
    return [r.as_dict() for r in res], Cs, Fs
