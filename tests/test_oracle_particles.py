"""Pins of the particle oracle: gather, Boris push, tet walk, quantised path-integral deposit.

Pinned against: the closed form of the Boris gyro-orbit and of the E x B drift, the
line integral of W1 computed by brute force (exact tet intervals found by testing every
tet, Gauss-Legendre inside each), brute-force point location, analytic specular
reflection, and the discrete continuity equation G^T g = Q^{n+1} - Q^n (Sec. IV.B.1: the
path integral makes continuity hold analytically; here it must hold bit for bit).
"""
import numpy as np
import pytest

import qh_inputs as qi
from oracle import particles as P
from oracle import whitney as W
from oracle.complex_ import LOCAL_EDGES, Complex
from oracle.whitney import Operators

S = 1 << P.F_BITS


def uniform_dofs(cx, E0, B0):
    x = cx.xyz
    e = (x[cx.edges[:, 1]] - x[cx.edges[:, 0]]) @ np.asarray(E0, float)
    fa, fb, fc = (x[cx.faces[:, k]] for k in range(3))
    b = 0.5 * np.cross(fb - fa, fc - fa) @ np.asarray(B0, float)
    return e, b


@pytest.fixture(scope="module")
def box8():
    m = qi.BoxMesh(8)
    cx = Complex(m.xyz, m.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    return m, cx, op, P.ParticleOracle(cx, op.Minv)


def brute_locate(cx, Minv, r, tol=1e-12):
    lam = Minv[:, :, 0][None] + np.einsum("tij,pj->pti", Minv[:, :, 1:], r)
    inside = lam.min(axis=2) >= -tol
    return inside, lam


def brute_line_integral(cx, Minv, r0, r1, n_gl=8):
    """int W1_e . dl over the straight path r0 -> r1, by exact tet intervals."""
    d = r1 - r0
    lam0 = Minv[:, :, 0] + Minv[:, :, 1:] @ r0
    dl = Minv[:, :, 1:] @ d
    out = np.zeros(cx.Ne)
    xg, wg = np.polynomial.legendre.leggauss(n_gl)
    for t in range(cx.Nt):
        lo, hi = 0.0, 1.0
        for i in range(4):
            if abs(dl[t, i]) < 1e-300:
                if lam0[t, i] < 0:
                    lo, hi = 1.0, 0.0
                continue
            s = -lam0[t, i] / dl[t, i]
            if dl[t, i] > 0:
                lo = max(lo, s)
            else:
                hi = min(hi, s)
        if hi - lo <= 1e-15:
            continue
        s = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
        r = r0[None] + s[:, None] * d[None]
        Mt = np.repeat(Minv[t][None], n_gl, axis=0)
        for k, le in enumerate(LOCAL_EDGES):
            w1 = W.w1_at(Mt, r, le)
            out[cx.tet_edges[t, k]] += 0.5 * (hi - lo) * np.sum(wg * (w1 @ d))
    return out


def test_path_integral_closed_form(box8):
    """int_seg W1_ab . dl = l_a(r0) l_b(r1) - l_a(r1) l_b(r0) inside one tet."""
    _, cx, op, _ = box8
    rng = np.random.default_rng(1)
    xg, wg = np.polynomial.legendre.leggauss(8)
    for t in rng.integers(0, cx.Nt, 20):
        Pt = cx.xyz[cx.tets[t]]
        r0, r1 = rng.dirichlet(np.ones(4)) @ Pt, rng.dirichlet(np.ones(4)) @ Pt
        M = op.Minv[t]
        l0, l1 = M[:, 0] + M[:, 1:] @ r0, M[:, 0] + M[:, 1:] @ r1
        s = 0.5 * (xg + 1)
        r = r0[None] + s[:, None] * (r1 - r0)[None]
        Mt = np.repeat(M[None], 8, axis=0)
        for (a, b) in LOCAL_EDGES:
            quad = 0.5 * np.sum(wg * (W.w1_at(Mt, r, (a, b)) @ (r1 - r0)))
            assert abs(quad - (l0[a] * l1[b] - l1[a] * l0[b])) < 1e-14


def test_deposit_equals_brute_force_line_integral(box8):
    """With E = B = 0 the path is straight; the integer current equals 2^{2F} times the
    brute-force line integral of W1 along it, to the quantisation bound."""
    m, cx, op, po = box8
    rng = np.random.default_rng(5)
    n = 40
    x0 = rng.uniform(0.3, 0.7, (n, 3))
    tet0 = m.locate_boxes(x0)
    v = rng.normal(0, 1.0, (n, 3)) * 0.05    # about half a cell per step at dt = 1
    e = np.zeros(cx.Ne)
    b = np.zeros(cx.Nf)
    for p in range(n):
        out = po.push(e, b, x0[p:p + 1], v[p:p + 1], tet0[p:p + 1], 0.0, 1.0, 1)
        assert out["wall_hits"] == 0
        ref = brute_line_integral(cx, op.Minv, x0[p], out["x"][0])
        got = out["g"].astype(np.float64) / S ** 2
        # each quantised end point moves lambda by <= 2^-F per coordinate
        assert np.abs(got - ref).max() < 8 * (out["crossings"] + 1) * 2.0 ** -P.F_BITS
        # charge: final W0 weights, sum exactly 2^{2F}
        assert out["Q"].sum() == S * S


def test_continuity_bitwise_with_crossings_and_walls(jitter4):
    """G^T g = Q^{n+1} - Q^n exactly, over steps with many crossings and wall hits."""
    m, cx, op = jitter4
    po = P.ParticleOracle(cx, op.Minv)
    parts = qi.make_particles(m, qi.CONFIGS["jitter4"])
    x, v, tet = (a.astype(np.float64) for a in parts["e"])
    tet = tet.astype(np.int64)
    rng = np.random.default_rng(0)
    e = rng.normal(0, 1e3, cx.Ne) * cx.edge_lengths()
    e[cx.wall_edge] = 0
    _, b = uniform_dofs(cx, (0, 0, 0), (0.02, -0.01, 0.1))
    L = po.quantize_points(x, tet)
    Q = np.zeros(cx.Nn, np.int64)
    for i in range(4):
        np.add.at(Q, cx.tets[tet, i], -S * L[:, i])
    tot_cross = tot_wall = 0
    for _ in range(5):
        out = po.push(e, b, x, v * 3e4, tet, -qi.QE / qi.ME, 1e-11, -1)
        v = out["v"] / 3e4
        assert np.array_equal(cx.G.T @ out["g"], out["Q"] - Q)
        x, tet, Q = out["x"], out["tet"], out["Q"]
        tot_cross += out["crossings"]
        tot_wall += out["wall_hits"]
        assert out["lost"] == 0
        assert (x >= -1e-12).all() and (x <= 1 + 1e-12).all()
    assert tot_cross > 1000 and tot_wall > 50


def test_walk_final_tet_matches_brute_force(jitter4):
    m, cx, op = jitter4
    po = P.ParticleOracle(cx, op.Minv)
    parts = qi.make_particles(m, qi.CONFIGS["jitter4"])
    x, v, tet = (a.astype(np.float64) for a in parts["e"])
    out = po.push(np.zeros(cx.Ne), np.zeros(cx.Nf), x[:300], v[:300] * 1e5, tet[:300], 0.0,
                  1e-11, -1)
    inside, lam = brute_locate(cx, op.Minv, out["x"])
    lam_own = lam[np.arange(300), out["tet"]]
    assert lam_own.min() > -1e-12          # the final tet holds the final point
    assert inside.any(axis=1).all()
    assert out["crossings"] > 100


def test_specular_reflection(box8):
    m, cx, op, po = box8
    x0 = np.array([[0.5, 0.3, 0.05]])
    v = np.array([[0.01, 0.02, -0.2]])
    out = po.push(np.zeros(cx.Ne), np.zeros(cx.Nf), x0, v, m.locate_boxes(x0), 0.0, 1.0, 1)
    expect = x0[0] + v[0]
    expect[2] = -expect[2]
    assert np.allclose(out["x"][0], expect, atol=1e-14)
    assert np.allclose(out["v"][0], v[0] * np.array([1, 1, -1]), atol=1e-15)
    assert out["wall_hits"] == 1
    assert np.array_equal(cx.G.T @ out["g"], out["Q"] - _q_of(po, cx, x0, m.locate_boxes(x0)))


def _q_of(po, cx, x, tet):
    L = po.quantize_points(x, tet)
    Q = np.zeros(cx.Nn, np.int64)
    for i in range(4):
        np.add.at(Q, cx.tets[np.asarray(tet), i], S * L[:, i])
    return Q


def test_boris_gyro_orbit_closed_form(box8):
    """Uniform B, E = 0: |v| conserved, rotation 2 atan(qB dt/2m) per step, positions on a
    circle of radius |v_perp| dt / (2 sin(theta/2))."""
    m, cx, op, po = box8
    Bz = 0.1
    e, b = uniform_dofs(cx, (0, 0, 0), (0, 0, Bz))
    qm = -qi.QE / qi.ME
    dt = 5e-12
    x = np.array([[0.5, 0.5, 0.5]])
    v = np.array([[2e6, 0.0, 1e5]])
    tet = m.locate_boxes(x)
    theta = 2 * np.arctan(abs(qm) * Bz * dt / 2)
    R = 2e6 * dt / (2 * np.sin(theta / 2))
    xs, vs = [x[0].copy()], [v[0].copy()]
    for _ in range(60):
        out = po.push(e, b, x, v, tet, qm, dt, -1)
        x, v, tet = out["x"], out["v"], out["tet"]
        xs.append(x[0].copy())
        vs.append(v[0].copy())
    xs, vs = np.array(xs), np.array(vs)
    speed = np.linalg.norm(vs, axis=1)
    assert np.allclose(speed, speed[0], rtol=1e-13)
    ang = np.arccos(np.clip(np.einsum("ij,ij->i", vs[1:-1, :2], vs[2:, :2])
                            / (np.linalg.norm(vs[1:-1, :2], axis=1) * np.linalg.norm(vs[2:, :2], axis=1)), -1, 1))
    assert np.allclose(ang, theta, rtol=1e-9)
    # circle through the orbit points (z drifts uniformly)
    p = xs[1:, :2]
    A = np.c_[2 * p, np.ones(len(p))]
    sol = np.linalg.lstsq(A, (p ** 2).sum(1), rcond=None)[0]
    c = sol[:2]
    rad = np.linalg.norm(p - c, axis=1)
    assert np.allclose(rad, R, rtol=1e-9)
    assert np.allclose(np.diff(xs[:, 2]), 1e5 * dt, rtol=1e-12)


def test_boris_exb_drift(box8):
    """Uniform E perpendicular to B: the mean velocity over whole gyrations is E x B / B^2."""
    m, cx, op, po = box8
    E0, B0 = np.array([2e3, 0, 0]), np.array([0, 0, 0.05])
    e, b = uniform_dofs(cx, E0, B0)
    qm = -qi.QE / qi.ME
    dt = 2e-12
    theta = 2 * np.arctan(abs(qm) * 0.05 * dt / 2)
    steps = int(round(10 * 2 * np.pi / theta))
    x = np.array([[0.5, 0.5, 0.5]])
    v = np.array([[0.0, 0.0, 0.0]])
    tet = m.locate_boxes(x)
    x0 = x.copy()
    for _ in range(steps):
        out = po.push(e, b, x, v, tet, qm, dt, -1)
        x, v, tet = out["x"], out["v"], out["tet"]
    drift = (x[0] - x0[0]) / (steps * dt)
    expect = np.cross(E0, B0) / (B0 @ B0)
    assert abs(drift[1] - expect[1]) < 2e-3 * abs(expect[1])


def test_quantize_sums_and_bounds(jitter4):
    m, cx, op = jitter4
    po = P.ParticleOracle(cx, op.Minv)
    x, _, tet = qi.make_particles(m, qi.CONFIGS["jitter4"])["e"]
    L = po.quantize_points(x.astype(np.float64), tet)
    assert (L.sum(1) == S).all() and (L >= 0).all() and (L <= S).all()
    lam = op.Minv[tet, :, 0] + np.einsum("pij,pj->pi", op.Minv[tet, :, 1:], x.astype(np.float64))
    assert np.abs(L / S - lam).max() <= 2.0 ** -P.F_BITS * 2


def test_integer_deposit_list_telescopes(jitter4):
    """Pieces chained through shared faces (Lambda carried by vertex id): G^T g equals the
    end-point charge minus the start-point charge, for random integer coordinates."""
    _, cx, op = jitter4
    po = P.ParticleOracle(cx, op.Minv)
    rng = np.random.default_rng(11)
    segs_t, l0s, l1s, zs = [], [], [], []
    Qs = np.zeros(cx.Nn, np.int64)
    Qe = np.zeros(cx.Nn, np.int64)

    def rand_lam(force=None):
        w = rng.dirichlet(np.ones(4))
        Lm = np.floor(w * S).astype(np.int64)
        if force is not None:
            Lm[force] = 0
        Lm[np.argmax(Lm)] += S - Lm.sum()
        return Lm

    for _ in range(200):
        z = int(rng.choice([-1, 1, 2]))
        t = int(rng.integers(cx.Nt))
        La = rand_lam()
        for i in range(4):
            Qs[cx.tets[t, i]] += z * S * La[i]
        for _hop in range(int(rng.integers(0, 5))):
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
        for i in range(4):
            Qe[cx.tets[t, i]] += z * S * Lend[i]
    g, _ = po.deposit_list(segs_t, l0s, l1s, zs, np.zeros(0), np.zeros((0, 4)), np.zeros(0))
    assert np.array_equal(cx.G.T @ g, Qe - Qs)


def test_gather_random_dofs_matches_whitney_sums(jitter4):
    """E = sum_e e_e W1_e(r) and B = sum_f b_f W2_f(r) (Sec. II.C) for random edge and face
    DOFs (no D b = 0: the face field is then affine in each tet) at random points of random tets
    of the jittered mesh: the C gather of the particle oracle against the Whitney sums of
    oracle.whitney, which the continuity and incidence tests pin, to 1e-13 of the field size."""
    m, cx, op = jitter4
    po = P.ParticleOracle(cx, op.Minv)
    rng = np.random.default_rng(21)
    e = rng.normal(0.0, 1e3, cx.Ne) * cx.edge_lengths()
    b = rng.normal(0.0, 1e-3, cx.Nf)
    n = 4000
    tet = rng.integers(0, cx.Nt, n)
    w = rng.dirichlet(np.ones(4), n)
    x = np.einsum("pi,pid->pd", w, cx.xyz[cx.tets[tet]])
    Ec, Bc = po.gather(e, b, x, tet)
    Ep = W.field_E(cx, op.Minv, e, tet, x)
    Bp = W.field_B(cx, op.Minv, b, tet, x)
    assert np.abs(Ec - Ep).max() <= 1e-13 * np.abs(Ep).max()
    assert np.abs(Bc - Bp).max() <= 1e-13 * np.abs(Bp).max()
    # the sums are not degenerate: every edge and face term moves the result
    e2 = e.copy()
    e2[cx.tet_edges[tet[0], 3]] += 1.0
    assert not np.allclose(po.gather(e2, b, x[:1], tet[:1])[0], Ec[:1], rtol=0, atol=1e-12)
    b2 = b.copy()
    b2[cx.tet_faces[tet[0], 2]] += 1e-3
    assert not np.allclose(po.gather(e, b2, x[:1], tet[:1])[1], Bc[:1], rtol=0, atol=1e-15)
