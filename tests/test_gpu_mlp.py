"""Learned-start kernels through the C ABI against the numpy oracle: pair
features, FP32 and BF16 forward, loss gradient and Adam step, and an SCF
started from a density."""
import numpy as np
import pytest

import synth
from oracle import mlp as M
from oracle import ri as R
from oracle import scf as S
from tests.gpu_common import need_gpu, problem, to_np, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    need_gpu()
    import paper_2407_19614_amd as P
    s = synth.config_system("n400")
    pr = P.RIProblem(s)
    pr.build_3c()
    mu, nu = to_np(pr.pairs)[: pr.n_pairs].T
    f_ref = M.pair_features(s, mu.astype(np.int64), nu.astype(np.int64))
    f_mean, f_std = f_ref.mean(0), f_ref.std(0) + 1e-3
    params = M.init_params(seed=7)
    return s, pr, f_ref, f_mean, f_std, params


def test_pair_features(setup):
    s, pr, f_ref, *_ = setup
    print("case: n400 pair features", flush=True)
    f = to_np(pr.pair_features())
    err = np.abs(f - f_ref) / (np.abs(f_ref) + 1e-6)
    assert err.max() < 2e-6, err.max()


def test_delta_features_and_density_change(setup):
    """Change features between two geometries of the walk against the oracle,
    and the change targets / start density against their definitions."""
    s, pr, *_ = setup
    print("case: n400 change features", flush=True)
    xyz0 = synth.random_walk(s.xyz, 1, 0.05, 2.0, seed=11)[1]
    rng = np.random.default_rng(4)
    Dp = rng.standard_normal((s.N, s.N))
    Dp = Dp + Dp.T
    mu, nu = to_np(pr.pairs)[: pr.n_pairs].T.astype(np.int64)
    g = to_np(pr.pair_delta_features(torch.tensor(xyz0, device="cuda"), torch.tensor(Dp, device="cuda")))
    g_ref = M.delta_features(s, xyz0, mu, nu, Dp)
    scale = np.maximum(np.abs(g_ref), 1e-3 * np.abs(g_ref).max(0))
    err = (np.abs(g - g_ref) / scale).max()
    print(f"max scaled |dg| = {err:.2e}", flush=True)
    assert err < 2e-6
    Dn = Dp + 1e-3 * rng.standard_normal((s.N, s.N))
    d = to_np(pr.density_change_pairs(torch.tensor(Dn, device="cuda"), torch.tensor(Dp, device="cuda"), 100.0))
    assert np.allclose(d, (100.0 * (Dn - Dp)[mu, nu]).astype(np.float32), rtol=1e-6, atol=1e-7)
    Dout = to_np(pr.density_add_pairs(torch.tensor(d, device="cuda"), 0.01, torch.tensor(Dp, device="cuda")))
    ref = Dp.copy()
    ref[mu, nu] = Dp[mu, nu] + 0.01 * d.astype(np.float64)
    ref[nu, mu] = ref[mu, nu]
    assert np.allclose(Dout, ref, rtol=1e-15, atol=1e-15)


def test_forward_fp32_bf16(setup):
    s, pr, f_ref, fm, fs, p = setup
    import paper_2407_19614_amd as P
    print("case: mlp forward", flush=True)
    net = P.MLP(P.pack_params(p), fm, fs)
    feat = torch.tensor(f_ref[:5000], dtype=torch.float32, device="cuda")
    x = (f_ref[:5000].astype(np.float32).astype(np.float64) - fm.astype(np.float32)) / fs.astype(np.float32)
    pp = P.unpack_params(P.pack_params(p))
    yref, _ = M.forward(pp, x)
    y32 = to_np(net.forward(feat, P.MLP_FP32))
    y16 = to_np(net.forward(feat, P.MLP_BF16))
    scale = np.abs(yref).max()
    print(f"fp32 max rel {np.abs(y32 - yref).max() / scale:.2e}  bf16 {np.abs(y16 - yref).max() / scale:.2e}")
    assert np.abs(y32 - yref).max() < 1e-5 * scale
    assert np.abs(y16 - yref).max() < 3e-2 * scale


def test_train_step_gradient_and_adam(setup):
    s, pr, f_ref, fm, fs, p = setup
    import paper_2407_19614_amd as P
    print("case: mlp train step", flush=True)
    net = P.MLP(P.pack_params(p), fm, fs)
    n = 3000
    rng = np.random.default_rng(3)
    t = rng.standard_normal(n).astype(np.float32) * 0.1
    feat = torch.tensor(f_ref[:n], dtype=torch.float32, device="cuda")
    loss, g = net.train_step(feat, torch.tensor(t, device="cuda"), lr=1e-3, want_grad=True)
    pp = P.unpack_params(P.pack_params(p))
    x = (f_ref[:n].astype(np.float32).astype(np.float64) - fm.astype(np.float32)) / fs.astype(np.float32)
    lref, gref = M.loss_and_grad(pp, x, t.astype(np.float64))
    assert abs(float(to_np(loss)[0]) - lref) < 1e-5 * lref
    gv = P.unpack_params(to_np(g))
    for k in gref:
        sc = np.abs(gref[k]).max()
        assert np.abs(gv[k] - gref[k]).max() < 1e-4 * sc + 1e-9, k
    m = {k: np.zeros_like(v) for k, v in pp.items()}
    v = {k: np.zeros_like(v) for k, v in pp.items()}
    newp = M.adam_step(pp, gref, m, v, 1, lr=1e-3)
    got = P.unpack_params(to_np(net.params))
    for k in newp:
        # first Adam step moves each weight by ~lr * sign(g); compare where |g| is not tiny
        sel = np.abs(gref[k]) > 1e-4 * np.abs(gref[k]).max()
        assert np.abs(got[k] - newp[k])[sel].max() < 2e-6, k


def test_energy_from_density_guess():
    need_gpu()
    import paper_2407_19614_amd as P
    print("case: tiny energy from density", flush=True)
    s = synth.config_system("tiny")
    ref = S.run_scf(s, R.RIData(s), tol_E=1e-12, tol_e=1e-10)
    pr = problem(s)
    D = torch.tensor(ref.D, dtype=torch.float64, device="cuda")
    res, C, F, Dg = pr.energy(tol_E=1e-12, tol_err=1e-9, guess_density=D)
    assert res["converged"] and res["n_iter"] <= 3
    assert abs(res["E_total"] - ref.E) < 1e-10
    # density scatter round trip over the pair list
    pairs = to_np(pr.pairs)[: pr.n_pairs]
    d = ref.D[pairs[:, 0], pairs[:, 1]].astype(np.float32)
    Dd = to_np(pr.density_from_pairs(torch.tensor(d, device="cuda")))
    assert np.abs(Dd[pairs[:, 0], pairs[:, 1]] - d).max() == 0 and np.abs(Dd - Dd.T).max() == 0
