"""Shared helpers for the GPU parity tests (inputs and device setup)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def problem(system, prec=0):
    import paper_2407_19614_amd as P
    pr = P.RIProblem(system, device="cuda", prec=prec)
    pr.build_3c()
    pr.metric_factor(prec)
    return pr


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
