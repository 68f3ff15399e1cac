"""Shared set-up for the GPU parity tests: the same seeded inputs go to the HIP path
(through the C ABI) and to the oracle. Nothing here computes the method."""
import numpy as np

import qh_inputs as qi

S = 1 << 20


def record(name, data):
    """Measured figures for the documentation (error tables), written as JSON when the
    environment variable QH_RECORD_DIR names a folder; nothing otherwise."""
    import json
    import os
    d = os.environ.get("QH_RECORD_DIR")
    if d:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, name + ".json"), "w") as fh:
            json.dump(data, fh, indent=1, default=float)


# FP32 unit roundoff and the bars derived from it for one FP32 gather and push against FP64
# (measured on the jittered 4^3 mesh and 4096 sampled 64^3 particles: at most 3 u for E and B,
# 2.3 u of the unit cube's extent for positions, 4 u for velocities):
#  - E = alpha + beta x (r - c) and B from FP32 records: the record's own rounding (a few u),
#    r - c formed in FP32 (u |r| against |r - c| ~ h/4: up to 8 u of the affine term); 32 u
#  - x + dt v and the reflection in FP32 inside the unit cube: half an ulp of 1 per operation plus
#    dt times the velocity's error; 16 u (metres, coordinates <= 1)
#  - Boris rotation and the two half kicks, about 20 FP32 operations; 32 u of max |v|
U32 = 2.0 ** -24
GATHER_REL = 32 * U32
PUSH_X_ABS = 16 * U32
PUSH_V_REL = 32 * U32


def err_stats(a):
    """max and 99th percentile of an array of errors."""
    a = np.asarray(a, np.float64).ravel()
    return {"max": float(a.max()) if a.size else 0.0, "p99": float(np.quantile(a, 0.99)) if a.size else 0.0,
            "n": int(a.size)}


def gpu_context(mesh, dt, weight=1.0, u_b=2.0 ** -56):
    import paper_2103_06737_amd as qh
    ctx = qh.Context(0)
    ctx.mesh_upload(mesh.xyz, mesh.tets)
    ctx.set_physics(qi.EPS0, qi.MU0, dt, qi.QE * weight * 2.0 ** -40, u_b)
    return ctx


def oracle_setup(mesh):
    from oracle.complex_ import Complex
    from oracle.particles import ParticleOracle
    from oracle.whitney import Operators
    cx = Complex(mesh.xyz, mesh.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    return cx, op, ParticleOracle(cx, op.Minv)


def oracle_fields(cx, cfg, u_b, seed=0):
    from oracle.field import init_fields
    return init_fields(cx, qi.white(cx.Ne, seed, 3), qi.white(cx.Ne, seed, 5), cfg["sigma_e"], cfg["bz"],
                       cfg["sigma_b"], u_b)


def node_charge(po, cx, x, tet, z):
    L = po.quantize_points(np.asarray(x, np.float64), np.asarray(tet, np.int64))
    Q = np.zeros(cx.Nn, np.int64)
    for i in range(4):
        np.add.at(Q, cx.tets[np.asarray(tet), i], z * S * L[:, i])
    return Q


def chained_segments(cx, count, seed):
    """Random chains of pieces through shared faces with integer coordinates summing to 2^20,
    carried by vertex id (the structure the walk produces)."""
    rng = np.random.default_rng(seed)
    segs_t, l0s, l1s, zs, pts_t, pts_l, pts_z = [], [], [], [], [], [], []

    def rand_lam(force=None):
        w = rng.dirichlet(np.ones(4))
        Lm = np.floor(w * S).astype(np.int64)
        if force is not None:
            Lm[force] = 0
        Lm[np.argmax(Lm)] += S - Lm.sum()
        return Lm

    for _ in range(count):
        z = int(rng.choice([-1, 1, 2]))
        t = int(rng.integers(cx.Nt))
        La = rand_lam()
        for _hop in range(int(rng.integers(0, 6))):
            k = int(rng.integers(4))
            nb = cx.tet_nbr[t, k]
            if nb < 0:
                break
            Lc = rand_lam(force=k)
            segs_t.append(t); l0s.append(La); l1s.append(Lc); zs.append(z)
            Ln = np.zeros(4, np.int64)
            for j in range(4):
                hit = np.flatnonzero(cx.tets[t] == cx.tets[nb, j])
                Ln[j] = Lc[hit[0]] if hit.size else 0
            t, La = nb, Ln
        Lend = rand_lam()
        segs_t.append(t); l0s.append(La); l1s.append(Lend); zs.append(z)
        pts_t.append(t); pts_l.append(Lend); pts_z.append(z)
    return (np.array(segs_t), np.array(l0s), np.array(l1s), np.array(zs),
            np.array(pts_t), np.array(pts_l), np.array(pts_z))
