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


class CylinderMesh:
    """Circular cylinder of radius R along z from 0 to L (the cavity of the beam test of
    Sec. VI.B), cut into tets.

    The disk is a centre node and nr concentric rings, ring k at radius R k / nr with 6k
    nodes at angles 2 pi j / (6k); two neighbouring rings are joined by walking both in
    angle order (6 nr^2 triangles). Layer l of the extrusion sits at z = L l / nz and node
    (disk node n, layer l) has id l * N2 + n. Each triangular prism (a < b < c on the disk)
    splits into (a_l, b_l, c_l, c_l+1), (a_l, b_l, b_l+1, c_l+1), (a_l, a_l+1, b_l+1, c_l+1):
    every quadrilateral side is cut along the diagonal from its lowest id, so neighbouring
    prisms agree. Tet vertices are listed in ascending id. bottom_tet[i] is the tet that
    holds disk triangle i of the z = 0 face.
    """

    def __init__(self, R: float, L: float, nr: int, nz: int):
        self.R, self.L, self.nr, self.nz = float(R), float(L), int(nr), int(nz)
        rings = [np.array([0])]
        xy = [(0.0, 0.0)]
        for k in range(1, nr + 1):
            m = 6 * k
            ang = 2.0 * np.pi * np.arange(m) / m
            rings.append(len(xy) + np.arange(m))
            r = R * k / nr
            xy += list(zip(r * np.cos(ang), r * np.sin(ang)))
        xy = np.array(xy)
        tri = [(0, 1 + j, 1 + (j + 1) % 6) for j in range(6)]
        for k in range(2, nr + 1):
            inner, outer = rings[k - 1], rings[k]
            n1, n2 = inner.size, outer.size
            i = j = 0
            while i < n1 or j < n2:
                # advance the ring whose next node comes first in angle
                a_next = (i + 1) / n1
                b_next = (j + 1) / n2
                if j < n2 and (i >= n1 or b_next <= a_next + 1e-12):
                    tri.append((inner[i % n1], outer[j % n2], outer[(j + 1) % n2]))
                    j += 1
                else:
                    tri.append((inner[i % n1], outer[j % n2], inner[(i + 1) % n1]))
                    i += 1
        tri = np.sort(np.array(tri, dtype=np.int64), axis=1)
        N2 = xy.shape[0]
        z = L * np.arange(nz + 1, dtype=np.float64) / nz
        self.xyz = np.concatenate([np.column_stack([xy, np.full(N2, zl)]) for zl in z])
        a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
        tets = []
        for l in range(nz):
            lo, hi = l * N2, (l + 1) * N2
            tets.append(np.stack([
                np.column_stack([a + lo, b + lo, c + lo, c + hi]),
                np.column_stack([a + lo, b + lo, b + hi, c + hi]),
                np.column_stack([a + lo, a + hi, b + hi, c + hi])], axis=1).reshape(-1, 4))
        self.tets = np.concatenate(tets).astype(np.int32)
        self.tri = tri
        self.n2 = N2
        self.bottom_tet = 3 * np.arange(tri.shape[0])   # (a_0, b_0, c_0, c_1) of layer 0

    def locate_bottom(self, p: np.ndarray) -> np.ndarray:
        """Disk triangle holding each point p (k x 2) of the z = 0 face (-1 if none)."""
        P = self.xyz[self.tri][:, :, :2]                      # (T, 3, 2)
        d = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
        det = d[0][:, 0] * d[1][:, 1] - d[0][:, 1] * d[1][:, 0]
        out = np.full(p.shape[0], -1, np.int64)
        for i, q in enumerate(p):
            r = q - P[:, 0]
            u = (r[:, 0] * d[1][:, 1] - r[:, 1] * d[1][:, 0]) / det
            w = (d[0][:, 0] * r[:, 1] - d[0][:, 1] * r[:, 0]) / det
            inside = np.flatnonzero((u >= -1e-12) & (w >= -1e-12) & (u + w <= 1.0 + 1e-12))
            if inside.size:
                out[i] = inside[0]
        return out

    def locate(self, p: np.ndarray) -> np.ndarray:
        """Tet holding each point p (k x 3) inside the cavity: its layer from z, its disk triangle,
        then the one of the prism's three tets whose barycentric coordinates are all >= 0 (up to
        rounding). -1 for a point outside."""
        p = np.asarray(p, np.float64)
        layer = np.clip((p[:, 2] / self.L * self.nz).astype(np.int64), 0, self.nz - 1)
        tri = self.locate_bottom(p[:, :2])
        out = np.full(p.shape[0], -1, np.int64)
        for i in np.flatnonzero(tri >= 0):
            best, tbest = -np.inf, -1
            for k in range(3):
                t = (layer[i] * self.tri.shape[0] + tri[i]) * 3 + k
                V = self.xyz[self.tets[t]]
                M = np.column_stack([V[1] - V[0], V[2] - V[0], V[3] - V[0]])
                l123 = np.linalg.solve(M, p[i] - V[0])
                lmin = min(1.0 - l123.sum(), l123.min())
                if lmin > best:
                    best, tbest = lmin, t
            if best > -1e-9:
                out[i] = tbest
        return out


def beam_injection_counts(steps: int, dt: float, per_step: float, t_on: float) -> np.ndarray:
    """Macro-particles injected in each of the first `steps` steps for a current that rises
    linearly from 0 to its full value over t_on and then stays (per_step particles per step
    at full current): differences of the rounded cumulative count."""
    t = dt * np.arange(steps + 1)
    rate = per_step / dt
    cum = np.where(t < t_on, 0.5 * rate * t * t / t_on, rate * (t - 0.5 * t_on))
    c = np.rint(cum).astype(np.int64)
    return np.diff(c)


def beam_injection(mesh: CylinderMesh, count: int, r_beam: float, v_p: float, seed: int = 0,
                   step: int = 0):
    """count electrons on the z = 0 face, uniform in the disk of radius r_beam, moving along
    +z at v_p (positions FP32, exactly on the face). Returns (x, v, tet)."""
    gen = rng(seed, 1000 + step)
    r = r_beam * np.sqrt(gen.random(count))
    phi = 2.0 * np.pi * gen.random(count)
    p = np.column_stack([r * np.cos(phi), r * np.sin(phi)]).astype(np.float32)
    tri = mesh.locate_bottom(p.astype(np.float64))
    assert (tri >= 0).all()
    x = np.column_stack([p, np.zeros(count, np.float32)]).astype(np.float32)
    v = np.zeros((count, 3), np.float32)
    v[:, 2] = v_p
    return x, v, mesh.bottom_tet[tri].astype(np.int32)


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


# Beam injected into a cylindrical PEC cavity (Sec. VI.B table): cavity radius 20 mm, length
# 100 mm; electrons at v_p = 5e7 m/s through the z = 0 face inside r_b = 8 mm; 10 macro-particles
# of 52012.58 electrons per step at the full 0.25 A, so dt = 10 * 52012.58 e / 0.25 A; the
# current turns on linearly over 2 ns; walls absorb. Mesh: 10 rings (2 mm), 50 layers (2 mm).
BEAM_CYL = dict(R=0.02, L=0.1, nr=10, nz=50, v_p=5e7, r_b=0.008, per_step=10, weight=52012.58,
                current=0.25, t_on=2e-9)
BEAM_CYL["dt"] = BEAM_CYL["per_step"] * BEAM_CYL["weight"] * QE / BEAM_CYL["current"]


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
