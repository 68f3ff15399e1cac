"""Pins of the field-update oracle (Sec. IV.B, Sec. V, Sec. VI.A).

  * the projected full-space trapezoidal update plus the Gauss-law solve equals the literal
    tree/co-tree reduced system built from Z11..Z23 exactly as printed (Sec. IV.B.2);
  * Z13 = 0 because Sigma = [*eps][grad] (Sec. IV.B.2);
  * the result does not depend on which spanning trees are used;
  * the source-free trapezoidal map has all eigenvalues on the unit circle (Sec. VI.A.1)
    and rotates each mode by 2 atan(omega dt / 2) (closed form of the trapezoidal rule);
  * the discrete energy is invariant without sources;
  * D b is invariant bit for bit (Sec. IV.A, Sec. V item 5);
  * Gauss's law holds after every step, and without the Gauss-law solve a loose Krylov
    tolerance leaves an error in it (Sec. I and Sec. V: the null space is excited to the
    level of the solver threshold).
"""
import json
import os

import numpy as np
import pytest

import qh_inputs as qi
from oracle import cotree as CT
from oracle import field as Fo

HERE = os.path.dirname(os.path.abspath(__file__))


def _exact_projected_step(cx, op, rs, dt, e, b, g, rho_new):
    ie, inn = rs.ie, rs.inn
    A = (op.Meps + dt * dt / 4 * op.S).toarray()[np.ix_(ie, ie)]
    Bm = (op.Meps - dt * dt / 4 * op.S).toarray()
    GtMe = (cx.G.T.astype(float) @ op.Meps).toarray()
    rhs = (Bm @ e + dt * (op.CtMmu @ b) - g)[ie]
    es = np.zeros(cx.Ne)
    es[ie] = np.linalg.solve(A, rhs)
    dl = np.linalg.solve(rs.K, rho_new - GtMe[inn] @ es)
    en = es.copy()
    en[ie] += rs.G @ dl
    bn = b - dt / 2 * (cx.C.astype(float) @ (en + e))
    return en, bn


def _source_free_state(cx, rs, seed=0):
    rng = np.random.default_rng(seed)
    e = np.zeros(cx.Ne)
    e[rs.ie] = rng.standard_normal(rs.ie.size)
    a = np.zeros(cx.Ne)
    a[rs.ie] = rng.standard_normal(rs.ie.size) * 1e-8
    b = cx.C.astype(float) @ a                     # zero flux through the PEC walls
    return e, b


@pytest.mark.parametrize("dt", [1e-11, 2e-9])
def test_literal_cotree_equals_projected(jitter4, dt):
    _, cx, op = jitter4
    rs = CT.ReducedSystem(cx, op, dt)
    e, b = _source_free_state(cx, rs)
    Ens, Es, Bs = rs.decompose(e[rs.ie], b[rs.jf])
    rho = rs.G.T @ rs.Me @ e[rs.ie]
    rng = np.random.default_rng(1)
    for _ in range(5):
        g = np.zeros(cx.Ne)
        g[rs.ie] = rng.standard_normal(rs.ie.size) * 1e-12
        rho_new = rho - rs.G.T @ g[rs.ie]          # continuity
        e, b = _exact_projected_step(cx, op, rs, dt, e, b, g, rho_new)
        Ens, Es, Bs = rs.step(Ens, Es, Bs, g[rs.ie], rho_new)
        rho = rho_new
        er, br = rs.compose(Ens, Es, Bs)
        assert np.abs(er - e[rs.ie]).max() <= 1e-10 * np.abs(e).max()
        assert np.abs(br - b[rs.jf]).max() <= 1e-10 * np.abs(b).max()


def test_z13_vanishes_and_square_blocks(jitter4):
    _, cx, op = jitter4
    rs = CT.ReducedSystem(cx, op, 1e-10)
    assert np.abs(rs.Z13).max() <= 1e-12 * np.abs(rs.Z12).max()
    assert rs.Z11.shape == rs.Z21.shape == (289, 289)


def test_tree_independence(jitter4):
    _, cx, op = jitter4
    dt = 1e-10
    outs = []
    for seed in (None, 5):
        rs = CT.ReducedSystem(cx, op, dt, tree_seed=seed)
        e, b = _source_free_state(cx, rs)
        Ens, Es, Bs = rs.decompose(e[rs.ie], b[rs.jf])
        rho = rs.G.T @ rs.Me @ e[rs.ie]
        g = np.random.default_rng(2).standard_normal(rs.ie.size) * 1e-12
        Ens, Es, Bs = rs.step(Ens, Es, Bs, g, rho - rs.G.T @ g)
        outs.append(rs.compose(Ens, Es, Bs))
    assert np.allclose(outs[0][0], outs[1][0], rtol=0, atol=1e-10 * np.abs(outs[0][0]).max())
    assert np.allclose(outs[0][1], outs[1][1], rtol=0, atol=1e-10 * np.abs(outs[0][1]).max())


def test_trapezoidal_map_unit_circle_and_phase(jitter4):
    _, cx, op = jitter4
    dt = 2e-9                                       # ~10x the explicit limit of this mesh
    ie = cx.int_edges
    jf = np.flatnonzero(~cx.wall_face)
    Me = op.Meps.toarray()[np.ix_(ie, ie)]
    Mm = op.Mmu.toarray()[np.ix_(jf, jf)]
    Cm = cx.C.toarray().astype(float)[np.ix_(jf, ie)]
    nf, ne = jf.size, ie.size
    M = np.block([[np.eye(nf), np.zeros((nf, ne))], [np.zeros((ne, nf)), Me]])
    H = np.block([[np.zeros((nf, nf)), -Cm], [Cm.T @ Mm, np.zeros((ne, ne))]])
    T = np.linalg.solve(M - 0.5 * dt * H, M + 0.5 * dt * H)
    mu = np.linalg.eigvals(T)
    assert np.abs(np.abs(mu) - 1).max() < 1e-10
    # phases: 2 atan(omega dt/2) with omega^2 the eigenvalues of [*eps]^-1 S
    S = Cm.T @ Mm @ Cm
    w2 = np.linalg.eigvals(np.linalg.solve(Me, S)).real
    w = np.sqrt(np.sort(w2[w2 > 1e-6 * w2.max()]))
    ph = np.sort(np.abs(np.angle(mu)))
    ph = ph[ph > 1e-8]
    expect = np.sort(np.concatenate([2 * np.arctan(w * dt / 2)] * 2))
    assert ph.size == expect.size
    assert np.allclose(ph, expect, rtol=1e-10, atol=1e-12)


def test_source_free_energy_and_divb(jitter4):
    _, cx, op = jitter4
    dt = 2e-9
    fo = Fo.FieldOracle(cx, op, dt)
    u_b = 2.0 ** -70
    rng = np.random.default_rng(3)
    e = np.zeros(cx.Ne)
    e[cx.int_edges] = rng.standard_normal(cx.int_edges.size)
    a = np.zeros(cx.Ne, np.int64)
    a[cx.int_edges] = rng.integers(-2 ** 40, 2 ** 40, cx.int_edges.size)
    b = cx.C @ a
    Db0 = cx.D @ b
    zero_n = np.zeros(cx.Nn, np.int64)
    rho0 = (fo.GtMeps @ e)[fo.inn]
    Qbg = np.zeros(cx.Nn, np.int64)

    def energy(e, b):
        br = b * u_b
        return e @ (op.Meps @ e) + br @ (op.Mmu @ br)

    W0 = energy(e, b)
    # keep the initial charge: rho = G^T [*eps] e^0 expressed through a background
    for _ in range(40):
        e, b, info = fo.step_with_rho(e, b, u_b, np.zeros(cx.Ne, np.int64), 1.0, rho0, tol=1e-13,
                                      tol_n=1e-13)
        assert np.array_equal(cx.D @ b, Db0)
    assert abs(energy(e, b) - W0) <= 1e-9 * W0


def test_gauss_law_and_qh_benefit(jitter4):
    """Loose edge solves (1e-6): with the Gauss-law solve the discrete Gauss residual stays
    at the nodal tolerance; without it the error is orders of magnitude larger."""
    m, cx, op = jitter4
    dt = 2e-9
    fo = Fo.FieldOracle(cx, op, dt)
    u_b = 2.0 ** -56
    rng = np.random.default_rng(4)
    e0 = np.zeros(cx.Ne)
    e0[cx.int_edges] = rng.standard_normal(cx.int_edges.size) * 1e2
    b0 = cx.C @ np.rint(rng.standard_normal(cx.Ne) * 1e-6 / u_b).astype(np.int64)
    u_q = 1e-12
    res = {}
    for gauss in (True, False):
        e, b = e0.copy(), b0.copy()
        Q = np.zeros(cx.Nn, np.int64)
        Qbg = np.zeros(cx.Nn, np.int64)
        errs = []
        r2 = np.random.default_rng(5)
        for _ in range(20):
            g = np.zeros(cx.Ne, np.int64)
            g[cx.int_edges] = r2.integers(-10 ** 6, 10 ** 6, cx.int_edges.size)
            Q = Q + cx.G.T @ g                       # continuity fixes the charge
            e, b, info = fo.step(e, b, u_b, g, u_q, Q, Qbg, tol=1e-6, tol_n=1e-12, gauss=gauss)
            rho = u_q * (Qbg - Q).astype(float)[fo.inn]
            errs.append(fo.gauss_error(e, rho))
        res[gauss] = np.array(errs)
    assert res[True][1:].max() < 1e-10
    assert res[False][1:].max() > 1e3 * res[True][1:].max()


def test_golden_beam_table_constants():
    """The beam table (Sec. VI.B) prints v_p = 5e7 m/s and v_p/c = 0.16678."""
    with open(os.path.join(HERE, "golden", "beam_table.json")) as f:
        gold = json.load(f)
    c = 1.0 / np.sqrt(qi.EPS0 * qi.MU0)
    assert abs(gold["v_p"] / c - gold["v_p_over_c"]) < 5e-6


def _wave_vs_trapezoidal(jitter4, tol, gauss, steps=20):
    """The trapezoidal (E-B) update from a Gauss-consistent start, and the wave-equation update
    started from its first two fields, driven by the same step currents."""
    m, cx, op = jitter4
    dt, u_b, u_q = 2e-9, 2.0 ** -56, 1e-12
    fo, wo = Fo.FieldOracle(cx, op, dt), Fo.WaveOracle(cx, op, dt)
    rng = np.random.default_rng(4)
    e0 = np.zeros(cx.Ne)
    e0[cx.int_edges] = rng.standard_normal(cx.int_edges.size) * 1e2
    e0 = fo.gauss_project(e0, np.zeros(cx.int_nodes.size), 1e-14, {})   # G^T [*eps] e0 = 0 = rho0
    b0 = cx.C @ np.rint(rng.standard_normal(cx.Ne) * 1e-6 / u_b).astype(np.int64)
    r2 = np.random.default_rng(5)
    gs = []
    for _ in range(steps):
        g = np.zeros(cx.Ne, np.int64)
        g[cx.int_edges] = r2.integers(-10 ** 6, 10 ** 6, cx.int_edges.size)
        gs.append(g)
    Qbg = np.zeros(cx.Nn, np.int64)
    e, b, Q = e0.copy(), b0.copy(), np.zeros(cx.Nn, np.int64)
    E_t, err_t = [e.copy()], []
    for k in range(steps):
        Q = Q + cx.G.T @ gs[k]
        e, b, info = fo.step(e, b, u_b, gs[k], u_q, Q, Qbg, tol=tol, tol_n=1e-12, gauss=gauss)
        E_t.append(e.copy())
        err_t.append(info["gauss_res"])
    Q = cx.G.T @ gs[0]
    ep, e, b = E_t[0].copy(), E_t[1].copy(), b0.copy()
    err_w, rel = [err_t[0]], []
    for k in range(1, steps):
        Q = Q + cx.G.T @ gs[k]
        rho = u_q * (Qbg - Q).astype(float)[wo.inn]
        en, b, info = wo.wave_step(e, ep, b, u_b, gs[k], gs[k - 1], u_q, rho, tol=tol, tol_n=1e-12, gauss=gauss)
        ep, e = e, en
        err_w.append(info["gauss_res"])
        rel.append(np.linalg.norm(e - E_t[k + 1]) / np.linalg.norm(E_t[k + 1]))
    return np.array(err_t), np.array(err_w), max(rel)


def test_wave_update_equals_trapezoidal(jitter4):
    """Newmark beta = 1/4 on the wave equation (eq. wave_cont) is the trapezoidal E-B update with
    b eliminated: from the same two first fields and currents the two sequences agree to the
    solver tolerance (tight solves: 1e-12)."""
    _, _, rel = _wave_vs_trapezoidal(jitter4, tol=1e-12, gauss=False)
    assert rel < 1e-9


def test_wave_gauss_error_grows_without_correction(jitter4):
    """Sec. V and the Gauss-law figure of Sec. VI: with loose solves (1e-6) and no correction the
    Gauss-law error of the E-B update levels off, that of the wave update grows step after
    step (the t grad Phi null space); with the correction both hold the law to the node
    solve's tolerance."""
    err_t, err_w, _ = _wave_vs_trapezoidal(jitter4, tol=1e-6, gauss=False)
    assert err_w[-1] > 5 * err_w[4] and err_w[-1] > 5 * err_t[-1]
    assert err_t[-1] < 2 * err_t[9]
    err_t, err_w, _ = _wave_vs_trapezoidal(jitter4, tol=1e-6, gauss=True)
    assert err_t.max() < 1e-10 and err_w.max() < 1e-10


def test_neumann_gauss_projection_zero_mean():
    """Natural boundary (eq. zero_mean_constraint): the Gauss-law system G^T[*eps]G on all nodes
    has the constants as null space; the projection solves it on the zero-mean subspace
    (alpha^T delta = 0, alpha_i the integral of W0_i) and reaches the law to its tolerance. e does
    not depend on the constant (G 1 = 0): the least-squares solution of the singular system gives
    the same field."""
    import scipy.sparse.linalg as sla
    from oracle.complex_ import Complex
    from oracle.whitney import Operators
    m = qi.make_mesh(qi.CONFIGS["jitter4"])
    cx = Complex(m.xyz, m.tets, neumann=True)
    op = Operators(cx, qi.EPS0, qi.MU0)
    fo = Fo.FieldOracle(cx, op, 2e-9)
    assert cx.int_edges.size == cx.Ne and cx.int_nodes.size == cx.Nn
    assert np.allclose(fo.K @ np.ones(cx.Nn), 0.0, atol=1e-12 * abs(fo.K).max())
    assert np.isclose(fo.alpha.sum(), 1.0)           # the unit cube's volume
    rng = np.random.default_rng(6)
    es = rng.standard_normal(cx.Ne) * 1e2
    q = rng.standard_normal(cx.Nn)
    rho = (q - q.mean()) * 1e-10                       # neutral: a consistent right-hand side
    info = {}
    e = fo.gauss_project(es, rho, 1e-13, info)
    assert fo.gauss_error(e, rho) < 1e-12
    dl = np.linalg.lstsq(fo.K.toarray(), fo.gauss_residual(es, rho), rcond=None)[0]
    e_ls = es + fo.Gint @ dl
    assert np.linalg.norm(e - e_ls) <= 1e-10 * np.linalg.norm(e)


def _plane_wave_run(n, gauss_flux=True, steps=100):
    from oracle.complex_ import Complex
    from oracle.whitney import Operators
    m = qi.BoxMesh(n, 1.0)
    cx = Complex(m.xyz, m.tets, neumann=True)
    op = Operators(cx, qi.EPS0, qi.MU0)
    f0, bw, dt = 150e6, 75e6, 0.1e-9
    fo = Fo.FieldOracle(cx, op, dt)
    pw = Fo.PlaneWave(cx, op, 1.0 / (2 * np.pi * f0), f0, bw, 4.0 / (2 * np.pi * bw))
    e, b = np.zeros(cx.Ne), np.zeros(cx.Nf, np.int64)
    g, d = np.zeros(cx.Ne, np.int64), np.zeros(cx.Nn)
    rel, gres = [], []
    for k in range(steps):
        hs = 0.5 * dt * (pw.h(k * dt) + pw.h((k + 1) * dt))
        if gauss_flux:
            d += fo.Gint.T @ hs
        e, b, info = fo.step_with_rho(e, b, 2.0 ** -56, g, 1.0, d, tol=1e-12, tol_n=1e-12, h_sum=hs)
        ref = pw.e_line((k + 1) * dt)
        rel.append(np.linalg.norm(e - ref) / np.linalg.norm(ref))
        gres.append(info["gauss_res"])
    return np.array(rel), np.array(gres)


def test_plane_wave_through_natural_boundary():
    """Sec. VI.A.2 with a resolved wave (150 MHz, 1 m box): n x H_inc imposed on every wall by
    the boundary term of Ampere's law drives the interior field to the incident plane wave
    (edge line integrals of E_inc), with second-order convergence (6^3 -> 8^3 boxes). The
    Gauss-law target carries the normal flux the wave brings in (G^T of the accumulated
    boundary term); with it the correction holds the law and keeps the field, without it the
    correction (rho = 0) spoils the field."""
    r6, g6 = _plane_wave_run(6)
    r8, g8 = _plane_wave_run(8)
    pk = slice(40, 70)                      # the pulse's main lobe is inside the box
    assert r6[pk].max() < 0.15 and r8[pk].max() < 0.7 * r6[pk].max()
    assert g6.max() < 1e-11 and g8.max() < 1e-11
    rb, _ = _plane_wave_run(6, gauss_flux=False)
    assert rb[pk].max() > 0.3


def test_plane_wave_face_subset():
    """The boundary term restricted to some wall faces equals the full one on every edge whose
    wall faces are all in the subset (the full-size GPU test samples edges this way)."""
    from oracle.complex_ import Complex
    from oracle.whitney import Operators
    m = qi.BoxMesh(4, 1.0)
    cx = Complex(m.xyz, m.tets, neumann=True)
    op = Operators(cx, qi.EPS0, qi.MU0)
    args = (1.0, 150e6, 75e6, 2e-9)
    full = Fo.PlaneWave(cx, op, *args)
    rng = np.random.default_rng(3)
    sample = rng.choice(np.flatnonzero(cx.wall_edge), 20, replace=False)
    faces = np.intersect1d(cx.C[:, sample].nonzero()[0], np.flatnonzero(cx.wall_face))
    part = Fo.PlaneWave(cx, op, *args, faces=faces)
    for t in (1.5e-9, 2e-9, 3e-9):
        hf, hp = full.h(t), part.h(t)
        assert (np.abs(hf[sample]) > 0).sum() >= 10   # zero on the y-walls (n x y-hat = 0)
        assert np.allclose(hp[sample], hf[sample], rtol=1e-13, atol=0)


def test_explicit_limit_is_the_leapfrog_stability_bound():
    """The explicit limit used to set the workloads' time steps, dt_CFL = 2 / sqrt(lambda_max
    ([*eps]^-1 S)), pinned twice: its eigenvalue agrees with a dense generalized symmetric
    eigen-solve, and it is the stability bound of the explicit leap-frog for [*eps] e'' = -S e
    (bounded just below it, exponential growth just above it)."""
    import scipy.linalg as sl
    from oracle.complex_ import Complex
    from oracle.whitney import Operators
    m = qi.BoxMesh(3)
    cx = Complex(m.xyz, m.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    dt = Fo.dt_cfl(op, cx, tol=1e-12)
    ie = cx.int_edges
    M = op.Meps[ie][:, ie].toarray()
    K = op.S[ie][:, ie].toarray()
    lam = sl.eigh(K, M, eigvals_only=True)
    assert abs(dt / (2.0 / np.sqrt(lam.max())) - 1) < 1e-8
    Minv_S = np.linalg.solve(M, K)
    rng = np.random.default_rng(0)

    def run(h, steps=600):
        e0 = rng.standard_normal(ie.size)
        e_prev, e = e0, e0.copy()
        top = 0.0
        for _ in range(steps):
            e_prev, e = e, 2 * e - e_prev - h * h * (Minv_S @ e)
            top = max(top, np.abs(e).max())
        return top / np.abs(e0).max()

    assert run(0.99 * dt) < 1e2
    assert run(1.01 * dt) > 1e6


def test_quasi_helmholtz_split():
    """E = grad(E_ns) + E_s (Sec. III): E_s has zero discrete divergence and is [*eps]-orthogonal
    to the potential part; the potential part has no curl; a gradient field is all E_ns, a field
    with [*eps] e in the range of C^T is all E_s; on a small mesh E_ns equals the literal
    projector form of the co-tree system; under natural walls E_ns has zero W0-weighted mean
    and E_s matches the PEC-free least-squares split."""
    from oracle.complex_ import Complex
    from oracle.cotree import ReducedSystem
    from oracle.whitney import Operators
    m = qi.make_mesh(qi.CONFIGS["jitter4"])
    cx = Complex(m.xyz, m.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    fo = Fo.FieldOracle(cx, op, 1e-10)
    rng = np.random.default_rng(11)
    e = np.zeros(cx.Ne)
    e[cx.int_edges] = rng.standard_normal(cx.int_edges.size)
    e_ns, e_s, rho = fo.decompose(e)
    Gf = cx.G.astype(float)
    div = (fo.GtMeps @ e_s)[cx.int_nodes]
    assert np.linalg.norm(div) <= 1e-11 * np.linalg.norm(rho)
    assert np.allclose(Gf @ e_ns + e_s, e, rtol=0, atol=1e-14 * np.abs(e).max())
    assert abs((Gf @ e_ns) @ (op.Meps @ e_s)) <= 1e-11 * np.sqrt((Gf @ e_ns) @ (op.Meps @ (Gf @ e_ns)) * (e_s @ (op.Meps @ e_s)))
    assert np.abs(cx.C @ (Gf @ e_ns)).max() <= 1e-13 * np.abs(e_ns).max()
    assert (e_ns[cx.wall_node] == 0).all()
    # pure gradient: all potential
    psi = np.zeros(cx.Nn)
    psi[cx.int_nodes] = rng.standard_normal(cx.int_nodes.size)
    g_ns, g_s, _ = fo.decompose(Gf @ psi)
    assert np.allclose(g_ns, psi, atol=1e-10) and np.abs(g_s).max() < 1e-10
    # [*eps] e = C^T w (zero discrete divergence): all solenoidal
    w = rng.standard_normal(cx.Nf)
    w[cx.wall_face] = 0.0
    ie = cx.int_edges
    e_c = np.zeros(cx.Ne)
    import scipy.sparse.linalg as sla
    e_c[ie] = sla.spsolve(op.Meps[ie][:, ie].tocsc(), (cx.C.T.astype(float) @ w)[ie])
    c_ns, c_s, _ = fo.decompose(e_c)
    assert np.abs(c_ns).max() <= 1e-10 * np.abs(e_c).max() / np.abs(Gf).max() and np.allclose(c_s, e_c, atol=1e-12 * np.abs(e_c).max())
    # the literal projector form (dense, co-tree system)
    rs = ReducedSystem(cx, op, 1e-10)
    Ens_lit, _, _ = rs.decompose(e[cx.int_edges], np.zeros(np.count_nonzero(~cx.wall_face)))
    assert np.allclose(e_ns[cx.int_nodes], Ens_lit, rtol=1e-9, atol=1e-12 * np.abs(Ens_lit).max())
    # natural walls: zero W0-weighted mean, same E_s as the least-squares solution of the singular system
    cn = Complex(m.xyz, m.tets, neumann=True)
    fn = Fo.FieldOracle(cn, op, 1e-10)
    en = rng.standard_normal(cn.Ne)
    n_ns, n_s, n_rho = fn.decompose(en)
    assert abs(fn.alpha @ n_ns) <= 1e-12 * np.abs(fn.alpha).sum() * np.abs(n_ns).max()
    phi_ls = np.linalg.lstsq(fn.K.toarray(), n_rho, rcond=None)[0]
    assert np.allclose(n_s, en - Gf @ phi_ls, atol=1e-9 * np.abs(en).max())
