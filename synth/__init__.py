"""Seeded synthetic inputs for the RI-HF hot path.

This module is shared by the CPU oracle and the HIP path, so it holds none of
the method's arithmetic: only random positions, exponent lists, index maps and
random matrices.  Every draw uses numpy's PCG64 through ``default_rng(seed)``.

The paper's workloads (polyglycine, water clusters, cc-pVDZ/def2 basis sets,
see its Results section) need p-g functions, fitting-basis data and geometries
that are not available; these clusters of helium-like centres carrying
even-tempered s-Gaussian bases stand in for them at the same N / N_aux sizes.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = ["System", "even_tempered", "cube_cluster", "ball_cluster",
           "make_system", "config_system", "random_walk", "random_coeffs",
           "batched_systems", "CONFIGS"]


@dataclasses.dataclass
class System:
    """Nuclei plus orbital and auxiliary s-Gaussian bases.

    Each basis function is one normalised primitive s-Gaussian.  Functions are
    ordered exponent-major: index = k * n_centres + centre, so that all
    functions of one exponent are contiguous.
    """
    xyz: np.ndarray          # [n_centres, 3] bohr
    Z: np.ndarray            # [n_centres]
    fn_centre: np.ndarray    # int32 [N]
    fn_exp: np.ndarray       # [N]
    aux_centre: np.ndarray   # int32 [N_aux]
    aux_exp: np.ndarray      # [N_aux]
    n_occ: int
    tau: float = 0.0         # pair screening threshold

    @property
    def n_centres(self):
        return self.xyz.shape[0]

    @property
    def N(self):
        return self.fn_exp.shape[0]

    @property
    def n_aux(self):
        return self.aux_exp.shape[0]

    def with_xyz(self, xyz):
        return dataclasses.replace(self, xyz=np.ascontiguousarray(xyz, dtype=np.float64))


def even_tempered(start: float, ratio: float, count: int) -> np.ndarray:
    return start * ratio ** np.arange(count, dtype=np.float64)


def _min_dist_ok(pts, p, dmin):
    if not pts:
        return True
    d = np.linalg.norm(np.asarray(pts) - p, axis=1)
    return bool(d.min() >= dmin)


def cube_cluster(n: int, side: float, dmin: float, seed: int) -> np.ndarray:
    """Uniform points in [0, side]^3, rejection sampling for min separation."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = rng.uniform(0.0, side, size=3)
        if _min_dist_ok(pts, p, dmin):
            pts.append(p)
    return np.asarray(pts, dtype=np.float64)


def ball_cluster(n: int, density: float, dmin: float, seed: int) -> np.ndarray:
    """Uniform points in a ball holding n centres at the given number density."""
    rng = np.random.default_rng(seed)
    radius = (3.0 * n / (4.0 * np.pi * density)) ** (1.0 / 3.0)
    pts = []
    while len(pts) < n:
        p = rng.uniform(-radius, radius, size=3)
        if np.dot(p, p) > radius * radius:
            continue
        if _min_dist_ok(pts, p, dmin):
            pts.append(p)
    return np.asarray(pts, dtype=np.float64)


def make_system(xyz, orb_exps, aux_exps, Zval=2.0, tau=0.0, n_occ=None) -> System:
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    nc = xyz.shape[0]
    orb_exps = np.asarray(orb_exps, dtype=np.float64)
    aux_exps = np.asarray(aux_exps, dtype=np.float64)
    fn_centre = np.tile(np.arange(nc, dtype=np.int32), orb_exps.size)
    fn_exp = np.repeat(orb_exps, nc)
    aux_centre = np.tile(np.arange(nc, dtype=np.int32), aux_exps.size)
    aux_exp = np.repeat(aux_exps, nc)
    Z = np.full(nc, float(Zval))
    if n_occ is None:
        n_occ = int(round(Z.sum())) // 2
    return System(xyz, Z, fn_centre, fn_exp, aux_centre, aux_exp, int(n_occ), float(tau))


# Per-centre bases of the five workloads.
ORB_TINY = np.array([0.3, 1.0, 3.5, 12.0])
AUX_TINY = even_tempered(0.1, 2.5, 10)
ORB_BIG = even_tempered(0.08, 2.2, 10)
AUX_BIG = even_tempered(0.05, 1.6, 30)

CONFIGS = {
    # 8 centres in a 10-bohr cube, N=32, N_aux=80, unscreened.
    "tiny": dict(kind="cube", n=8, side=10.0, dmin=2.5, seed=1, orb=ORB_TINY, aux=AUX_TINY, tau=0.0),
    # 100 centres at 0.01 / bohr^3, N=1000, N_aux=3000, tau=1e-12.
    "n1000": dict(kind="ball", n=100, density=0.01, dmin=2.5, seed=2, orb=ORB_BIG, aux=AUX_BIG, tau=1e-12),
    # 40 centres (N=400, N_aux=1200): start geometry of the geometry-sequence workload.
    "n400": dict(kind="ball", n=40, density=0.01, dmin=2.5, seed=5, orb=ORB_BIG, aux=AUX_BIG, tau=1e-12),
}


def config_system(name: str, n_centres: int | None = None, seed: int | None = None) -> System:
    c = dict(CONFIGS[name])
    if n_centres is not None:
        c["n"] = n_centres
    if seed is not None:
        c["seed"] = seed
    if c["kind"] == "cube":
        xyz = cube_cluster(c["n"], c["side"], c["dmin"], c["seed"])
    else:
        xyz = ball_cluster(c["n"], c["density"], c["dmin"], c["seed"])
    return make_system(xyz, c["orb"], c["aux"], tau=c["tau"])


def batched_systems(n_mol: int = 256, lo: int = 10, hi: int = 60, seed: int = 4000):
    """Uneven batch: n_centres ~ U{lo..hi}, seeds seed+k, config-2 bases."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=n_mol)
    out = []
    for k, nc in enumerate(sizes):
        xyz = ball_cluster(int(nc), 0.01, 2.5, seed + 1 + k)
        out.append(make_system(xyz, ORB_BIG, AUX_BIG, tau=1e-12))
    return out


def random_walk(xyz0, n_steps: int, sigma: float, dmin: float, seed: int):
    """Gaussian random walk of all coordinates; steps that bring any pair
    below dmin are redrawn.  Returns [n_steps + 1, n, 3]."""
    rng = np.random.default_rng(seed)
    cur = np.array(xyz0, dtype=np.float64)
    traj = [cur.copy()]
    iu = np.triu_indices(cur.shape[0], 1)
    for _ in range(n_steps):
        while True:
            nxt = cur + rng.normal(0.0, sigma, size=cur.shape)
            d = np.linalg.norm(nxt[:, None, :] - nxt[None, :, :], axis=-1)[iu]
            if d.min() >= dmin:
                break
        cur = nxt
        traj.append(cur.copy())
    return np.asarray(traj)


def random_coeffs(N: int, n_occ: int, seed: int) -> np.ndarray:
    """Seeded random occupied-coefficient block [N, n_occ] (row-major)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, n_occ)) / np.sqrt(N)
