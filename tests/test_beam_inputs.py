"""CPU tests of the cylindrical cavity, the beam injector (Sec. VI.B table) and the oracle's
absorbing walls."""
import numpy as np

import qh_inputs as qi


def _mesh():
    c = qi.BEAM_CYL
    return qi.CylinderMesh(c["R"], c["L"], c["nr"], c["nz"])


def test_cylinder_mesh_is_a_conforming_cavity():
    from oracle.complex_ import Complex
    c = qi.BEAM_CYL
    m = _mesh()
    P = m.xyz[m.tets]
    vol = np.einsum("ti,ti->t", P[:, 1] - P[:, 0], np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0])) / 6
    # the prism over the 6 nr-gon inscribed in the circle, filled without overlap
    ngon = 0.5 * 6 * c["nr"] * c["R"] ** 2 * np.sin(2 * np.pi / (6 * c["nr"]))
    assert np.abs(vol).min() > 0.1 * np.abs(vol).max()
    assert np.isclose(np.abs(vol).sum(), ngon * c["L"], rtol=1e-12)
    cx = Complex(m.xyz, m.tets)
    assert cx.Nn - cx.Ne + cx.Nf - cx.Nt == 1
    # two end caps, and the side: one quadrilateral (two triangles) per outer segment and layer
    assert cx.wall_face.sum() == 2 * m.tri.shape[0] + 2 * 6 * c["nr"] * c["nz"]
    w = m.xyz[cx.wall_node]
    r = np.hypot(w[:, 0], w[:, 1])
    on_surface = np.isclose(r, c["R"]) | np.isclose(w[:, 2], 0.0) | np.isclose(w[:, 2], c["L"])
    assert on_surface.all()
    el = np.linalg.norm(m.xyz[cx.edges[:, 0]] - m.xyz[cx.edges[:, 1]], axis=1)
    assert 1.9e-3 < el.min() and el.max() < 4.1e-3
    # the tet listed for each bottom triangle holds that triangle as a face
    for i in range(0, m.tri.shape[0], 37):
        assert set(m.tri[i]) <= set(m.tets[m.bottom_tet[i]])


def test_beam_injection_on_the_face_inside_the_beam():
    m = _mesh()
    x, v, tet = qi.beam_injection(m, 500, qi.BEAM_CYL["r_b"], qi.BEAM_CYL["v_p"], seed=0, step=3)
    assert x.dtype == np.float32 and (x[:, 2] == 0).all()
    assert (np.hypot(x[:, 0], x[:, 1]) <= qi.BEAM_CYL["r_b"] * (1 + 1e-6)).all()
    assert (v[:, 2] == np.float32(5e7)).all() and (v[:, :2] == 0).all()
    # each point lies in its tet (barycentric coordinates of the bottom face, fourth zero)
    from oracle.complex_ import Complex
    from oracle.whitney import Operators
    cx = Complex(m.xyz, m.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    lam = np.einsum("tij,tj->ti", op.Minv[tet], np.column_stack([np.ones(500), x.astype(np.float64)]))
    assert lam.min() > -1e-9
    # fewer particles while the current turns on, then per_step every step; the counts add up
    # to the charge the current carried
    c = qi.BEAM_CYL
    n = qi.beam_injection_counts(9000, c["dt"], c["per_step"], c["t_on"])
    ramp = int(round(c["t_on"] / c["dt"]))
    assert (n[ramp + 5:] == c["per_step"]).all() and n[:100].sum() < 20
    q = n.sum() * c["weight"] * qi.QE
    t = 9000 * c["dt"]
    assert abs(q - c["current"] * (t - 0.5 * c["t_on"])) <= c["weight"] * qi.QE


def test_oracle_absorbing_walls():
    """A particle that reaches a wall stops at the wall point: the path up to it is deposited,
    its charge is not; continuity then holds on every node off the walls (the charge leaves
    through the wall), and on the walls the deposit differs by the charge that left."""
    from oracle.complex_ import Complex
    from oracle.particles import ParticleOracle
    from oracle.whitney import Operators
    m = _mesh()
    cx = Complex(m.xyz, m.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    po = ParticleOracle(cx, op.Minv)
    gen = np.random.default_rng(2)
    k = 200
    # points near the side wall moving outward, near the far end moving +z, and inside
    phi = 2 * np.pi * gen.random(k)
    r = np.where(np.arange(k) % 2 == 0, 0.0185, 0.01 * gen.random(k))
    z = np.where(np.arange(k) % 2 == 0, 0.05, 0.099)
    x = np.column_stack([r * np.cos(phi), r * np.sin(phi), z])
    vr = np.where(np.arange(k) % 2 == 0, 2e7, 0.0)
    v = np.column_stack([vr * np.cos(phi), vr * np.sin(phi), np.where(np.arange(k) % 2 == 0, 0.0, 3e7)])
    v[::10] *= 0.01    # a few stay inside
    # locate: brute force over tets
    lam = np.einsum("tij,pj->pti", op.Minv, np.column_stack([np.ones(k), x]))
    tet = np.argmax(lam.min(axis=2), axis=1)
    dt = 1e-10
    zq = -1
    L0 = po.quantize_points(x, tet)
    _, Q0 = po.deposit_list(np.zeros(0), np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0), tet, L0, np.full(k, zq))
    out = po.push(np.zeros(cx.Ne), np.zeros(cx.Nf), x, v, tet, -qi.QE / qi.ME, dt, zq, absorb=True)
    gone = out["absorbed"]
    assert 50 < gone.sum() < k - 10 and out["lost"] == 0
    # absorbed particles end on the cavity surface
    xe = out["x"][gone]
    re = np.hypot(xe[:, 0], xe[:, 1])
    on_wall = (re > 0.0199 * np.cos(np.pi / 60)) | np.isclose(xe[:, 2], 0.1)
    assert on_wall.all()
    d = cx.G.T @ out["g"] - (out["Q"] - Q0)
    assert (d[~cx.wall_node] == 0).all()
    assert (d[cx.wall_node] != 0).any()
    # the difference on the walls is the charge the absorbed particles took out, at their
    # wall points (quantised there with the coordinate opposite the wall face at zero)
    S = 1 << 20
    assert d.sum() == zq * S * S * gone.sum()
    # without absorption every particle stays and continuity holds everywhere
    out_r = po.push(np.zeros(cx.Ne), np.zeros(cx.Nf), x, v, tet, -qi.QE / qi.ME, dt, zq)
    assert not out_r["absorbed"].any()
    assert (cx.G.T @ out_r["g"] == out_r["Q"] - Q0).all()
