"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module only draws random numbers and lays out synthetic meshes and particle
clouds. It holds none of the method's arithmetic (no Whitney forms, no operators,
no push, walk or deposit): both sides receive the same arrays and compute from them
independently.

Meshes are cubes [0,L]^3 cut into n^3 boxes, each box split into the six tetrahedra
that follow the monotone lattice paths from its lowest to its highest corner (Kuhn
split). The paper meshes its domains with an unstructured mesher (Sec. VI); these
meshes stand in for them with the sizes of the workloads.
"""
from __future__ import annotations

import itertools

import numpy as np

# Kuhn permutations in a fixed order: tet 6*c + p of box c follows the path
# e_{pi[0]}, e_{pi[1]}, e_{pi[2]}.
PERMS = list(itertools.permutations((0, 1, 2)))

# CODATA-2018 constants (SI)
EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6
QE = 1.602176634e-19
ME = 9.1093837015e-31
MI = 1836.0 * ME


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """PCG64 generator for (seed, stream); streams keep draws independent."""
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


def graded_grid(n: int, L: float, ratio: float) -> np.ndarray:
    """n+1 coordinates in [0,L] with spacings h_k = h0*ratio^k (k = 0..n-1)."""
    if ratio == 1.0:
        g = L * np.arange(n + 1, dtype=np.float64) / n
    else:
        h0 = L * (ratio - 1.0) / (ratio ** n - 1.0)
        h = h0 * ratio ** np.arange(n, dtype=np.float64)
        g = np.concatenate([[0.0], np.cumsum(h)])
    g[-1] = L
    return g


class BoxMesh:
    """Kuhn-split box mesh: node coordinates and tet connectivity.

    Node id = i + (n+1)*(j + (n+1)*k). Tet id = 6*(i + n*(j + n*k)) + p, with p the
    index of the permutation in PERMS. Vertices of every tet are listed along its
    lattice path, which is also ascending node id.
    """

    def __init__(self, n: int, L: float = 1.0, jitter: float = 0.0,
                 z_ratio: float = 1.0, seed: int = 0):
        self.n, self.L = int(n), float(L)
        self.gx = graded_grid(n, L, 1.0)
        self.gy = graded_grid(n, L, 1.0)
        self.gz = graded_grid(n, L, z_ratio)
        n1 = n + 1
        i, j, k = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
        i, j, k = (a.transpose(2, 1, 0).ravel() for a in (i, j, k))  # node id order
        xyz = np.stack([self.gx[i], self.gy[j], self.gz[k]], axis=1)
        self.jittered = jitter > 0.0
        if self.jittered:
            interior = (i > 0) & (i < n) & (j > 0) & (j < n) & (k > 0) & (k < n)
            h = L / n
            d = rng(seed, 1).uniform(-jitter * h, jitter * h, size=(int(interior.sum()), 3))
            xyz[interior] += d
        self.xyz = xyz
        ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        ci, cj, ck = (a.transpose(2, 1, 0).ravel() for a in (ci, cj, ck))
        base = np.stack([ci, cj, ck], axis=1)
        tets = np.empty((n ** 3, 6, 4), dtype=np.int64)
        for p, perm in enumerate(PERMS):
            v = base.copy()
            tets[:, p, 0] = v[:, 0] + n1 * (v[:, 1] + n1 * v[:, 2])
            for m in range(3):
                v[:, perm[m]] += 1
                tets[:, p, m + 1] = v[:, 0] + n1 * (v[:, 1] + n1 * v[:, 2])
        self.tets = tets.reshape(-1, 4).astype(np.int32)

    @property
    def n_nodes(self) -> int:
        return self.xyz.shape[0]

    @property
    def n_tets(self) -> int:
        return self.tets.shape[0]

    def locate_boxes(self, pos: np.ndarray) -> np.ndarray:
        """Tet ids of points in an unjittered mesh (box index, then Kuhn permutation)."""
        assert not self.jittered
        n = self.n
        idx, frac = [], []
        for a, g in enumerate((self.gx, self.gy, self.gz)):
            c = np.clip(np.searchsorted(g, pos[:, a], side="right") - 1, 0, n - 1)
            idx.append(c)
            frac.append((pos[:, a] - g[c]) / (g[c + 1] - g[c]))
        frac = np.stack(frac, axis=1)
        order = np.argsort(-frac, axis=1, kind="stable")
        perm_id = np.zeros(pos.shape[0], dtype=np.int64)
        for p, perm in enumerate(PERMS):
            perm_id[np.all(order == np.array(perm), axis=1)] = p
        cell = idx[0] + n * (idx[1] + n * idx[2])
        return (6 * cell + perm_id).astype(np.int32)

    def sample_uniform_by_tet(self, count: int, gen: np.random.Generator):
        """Points uniform in the domain: tet drawn by volume, then uniform barycentrics."""
        P = self.xyz[self.tets]
        vol = np.abs(np.einsum("ti,ti->t", P[:, 1] - P[:, 0],
                               np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0])))
        t = gen.choice(self.n_tets, size=count, p=vol / vol.sum())
        u = np.sort(gen.random((count, 3)), axis=1)
        w = np.diff(np.concatenate([np.zeros((count, 1)), u, np.ones((count, 1))], axis=1), axis=1)
        pos = np.einsum("pi,pid->pd", w, P[t])
        return pos, t.astype(np.int32)


def maxwellian(count: int, v_th: float, gen: np.random.Generator, drift=(0.0, 0.0, 0.0)):
    v = gen.normal(0.0, v_th, size=(count, 3))
    v += np.asarray(drift, dtype=np.float64)
    return v


def uniform_plasma(mesh: BoxMesh, count: int, v_th: float, seed: int = 0, stream: int = 2):
    """Uniform positions and a Maxwellian (per-component std v_th); float32 out."""
    gen = rng(seed, stream)
    if mesh.jittered:
        pos, tet = mesh.sample_uniform_by_tet(count, gen)
    else:
        pos = gen.random((count, 3)) * mesh.L
        tet = mesh.locate_boxes(pos)
    vel = maxwellian(count, v_th, gen)
    return pos.astype(np.float32), vel.astype(np.float32), tet


def beam(mesh: BoxMesh, count: int, sigma_frac: float, drift_z: float, v_th: float,
         seed: int = 0, stream: int = 2):
    """Gaussian beam along z: transverse N(L/2, (sigma_frac*L)^2) redrawn until inside,
    z uniform, drift along +z plus a thermal spread."""
    gen = rng(seed, stream)
    L = mesh.L
    xy = np.empty((count, 2))
    todo = np.arange(count)
    while todo.size:
        d = gen.normal(0.5 * L, sigma_frac * L, size=(todo.size, 2))
        ok = np.all((d > 0.0) & (d < L), axis=1)
        xy[todo[ok]] = d[ok]
        todo = todo[~ok]
    z = gen.random(count) * L
    pos = np.concatenate([xy, z[:, None]], axis=1)
    tet = mesh.locate_boxes(pos)
    vel = maxwellian(count, v_th, gen, drift=(0.0, 0.0, drift_z))
    return pos.astype(np.float32), vel.astype(np.float32), tet


def white(count: int, seed: int = 0, stream: int = 3) -> np.ndarray:
    """Standard-normal float64 draws (per-DOF random field amplitudes)."""
    return rng(seed, stream).standard_normal(count)


# Workloads -----------------------------------------------------------------

CONFIGS = {
    # jittered 4^3 Kuhn cube, 1,000 electrons, full cycle, 100 steps
    "jitter4": dict(n=4, jitter=0.1, z_ratio=1.0, n_e=1000, n_i=0, v_th_e=1e6, v_th_i=0.0,
               weight=1.0, dt=1e-11, steps=100, sigma_e=1e3, bz=0.1, sigma_b=0.0,
               mode="solve", load="uniform"),
    # 32^3, 1M-electron beam in frozen random fields, 200 steps
    "beam32": dict(n=32, jitter=0.0, z_ratio=1.0, n_e=1_000_000, n_i=0, v_th_e=1e5, v_th_i=0.0,
               weight=1.0, dt=1e-11, steps=200, sigma_e=1e4, bz=0.1, sigma_b=1e-3,
               mode="frozen", load="beam", beam_sigma=0.1, drift_z=1e7),
    # 64^3, 16M-electron uniform plasma (n = 1e16 m^-3), full cycle at 10x the explicit
    # limit (dt_CFL(64^3) ~ 1.20e-11 s from the oracle's eigen-analysis, oracle/cfl.py)
    "plasma64": dict(n=64, jitter=0.0, z_ratio=1.0, n_e=16_000_000, n_i=0, v_th_e=1e6, v_th_i=0.0,
               weight=1e16 / 16_000_000, dt=1.2e-10, steps=100, sigma_e=0.0, bz=0.1,
               sigma_b=0.0, mode="solve", load="uniform", sort_every=20),
    # 96^3 graded toward z = 0 (ratio 1.05), 32M electrons + 32M ions, full cycle at 10x the
    # explicit limit. dt_CFL: the oracle's eigen-analysis of a 16^3 mesh graded to the same
    # thinnest-cell aspect (22:1, ratio 1.35) gives n * dt_CFL = 5.32e-10 s, so ~5.5e-12 s at
    # n = 96 (the thin layers cost only a factor 1.45 against the uniform lattice).
    "graded96": dict(n=96, jitter=0.0, z_ratio=1.05, n_e=32_000_000, n_i=32_000_000, v_th_e=1e6,
               v_th_i=2e4, weight=1e16 / 32_000_000, dt_cfl_mult=10.0, dt=5.5e-11, steps=200,
               sigma_e=0.0, bz=0.1, sigma_b=0.0, mode="solve", load="uniform", sort_every=20),
}


def make_mesh(cfg: dict, seed: int = 0) -> BoxMesh:
    return BoxMesh(cfg["n"], 1.0, jitter=cfg.get("jitter", 0.0),
                   z_ratio=cfg.get("z_ratio", 1.0), seed=seed)


def make_particles(mesh: BoxMesh, cfg: dict, seed: int = 0, n_e: int | None = None):
    """Electron cloud (and an ion cloud on the same positions when the workload has ions)."""
    n_e = cfg["n_e"] if n_e is None else n_e
    if cfg.get("load") == "beam":
        pos, vel, tet = beam(mesh, n_e, cfg["beam_sigma"], cfg["drift_z"], cfg["v_th_e"], seed)
    else:
        pos, vel, tet = uniform_plasma(mesh, n_e, cfg["v_th_e"], seed)
    out = {"e": (pos, vel, tet)}
    if cfg.get("n_i", 0):
        gi = rng(seed, 4)
        vel_i = maxwellian(n_e, cfg["v_th_i"], gi).astype(np.float32)
        out["i"] = (pos.copy(), vel_i, tet.copy())
    return out
