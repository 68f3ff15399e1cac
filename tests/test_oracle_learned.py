"""Pins of the learned-preconditioner oracle.

  * the hand-written backward pass matches central finite differences of the loss;
  * a network that outputs zero gives exactly the Jacobi preconditioner (same PCG iterates
    as the plain solver);
  * with the exact trace the loss is log K >= 0 (Kaporin number, AM-GM), and K = 1 for the
    inverse Cholesky factor of A;
  * training lowers the loss and cuts PCG iterations to 1e-8 on held-out right-hand sides.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import qh_inputs as qi
from oracle import field as Fo
from oracle import learned as Lr
from oracle.complex_ import Complex
from oracle.whitney import Operators


def edge_problem(n, cfl_mult=10.0, jitter=0.0):
    m = qi.BoxMesh(n, jitter=jitter)
    cx = Complex(m.xyz, m.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    dt = cfl_mult * 7.69e-10 / n
    tau = dt * dt / 4
    ie = cx.int_edges
    A = (op.Meps + tau * op.S)[ie][:, ie].tocsr()
    Me = op.Meps[ie][:, ie].tocsr()
    S = op.S[ie][:, ie].tocsr()
    ev = (cx.xyz[cx.edges[:, 1]] - cx.xyz[cx.edges[:, 0]])[ie]
    rows, cols = Lr.lower_pattern(A)
    f = Lr.features(A, Me, S, tau, ev, rows, cols)
    return A, rows, cols, f


@pytest.fixture(scope="module")
def small():
    return edge_problem(3, jitter=0.1)


def _random_weights(seed):
    w = Lr.init_weights(seed)
    rng = np.random.default_rng(seed + 1)
    w["W3"] = rng.normal(0, 0.05, w["W3"].shape)
    w["b1"] = rng.normal(0, 0.1, w["b1"].shape)
    w["b2"] = rng.normal(0, 0.1, w["b2"].shape)
    return w


def test_gradient_matches_finite_differences(small):
    A, rows, cols, f = small
    w = _random_weights(3)
    V = np.sign(np.random.default_rng(5).standard_normal((A.shape[0], 4)))
    L, g, _ = Lr.kaporin_loss_grad(w, A, f, rows, cols, V)
    rng = np.random.default_rng(7)
    for _ in range(4):
        d = {k: rng.standard_normal(v.shape) for k, v in w.items()}
        h = 1e-6
        wp = {k: w[k] + h * d[k] for k in w}
        wm = {k: w[k] - h * d[k] for k in w}
        Lp = Lr.kaporin_loss_grad(wp, A, f, rows, cols, V)[0]
        Lm = Lr.kaporin_loss_grad(wm, A, f, rows, cols, V)[0]
        fd = (Lp - Lm) / (2 * h)
        an = sum(np.sum(g[k] * d[k]) for k in w)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_zero_network_is_jacobi(small):
    A, rows, cols, f = small
    w = Lr.init_weights(0)                 # last layer zero
    o, _ = Lr.mlp_forward(w, f)
    assert not o.any()
    G, _ = Lr.factor(o, rows, cols, A.diagonal(), A.shape[0])
    M = (G.T @ G).toarray()
    assert np.allclose(M, np.diag(1.0 / A.diagonal()), rtol=1e-14, atol=0)
    b = A @ np.random.default_rng(1).standard_normal(A.shape[0])
    x1, it1 = Lr.pcg(A, b, lambda r: G.T @ (G @ r), tol=1e-10)
    x2, it2, _ = Fo.pcg(A, b, tol=1e-10)
    assert abs(it1 - it2) <= 1 and np.allclose(x1, x2, rtol=1e-8)   # rounding of D^-1/2 D^-1/2 vs D^-1


def test_kaporin_bounds(small):
    A, rows, cols, f = small
    n = A.shape[0]
    logdetA = np.linalg.slogdet(A.toarray())[1]
    I = np.eye(n)
    for seed in range(3):
        w = _random_weights(seed)
        o, _ = Lr.mlp_forward(w, f)
        _, vals = Lr.factor(o, rows, cols, A.diagonal(), n)
        L, _ = Lr.kaporin_loss_grad_G(A, rows, cols, vals, I)   # exact trace
        assert L - logdetA / n >= -1e-12          # log K = L - log det(A) / n
    # the inverse Cholesky factor (full lower pattern) reaches K = 1
    Ad = A.toarray()
    Linv = np.linalg.inv(np.linalg.cholesky(Ad))
    r, c = np.tril_indices(n)
    L, _ = Lr.kaporin_loss_grad_G(sp.csr_matrix(Ad), r, c, Linv[r, c], I)
    assert abs(L - logdetA / n) < 1e-9


@pytest.mark.slow
def test_training_cuts_pcg_iterations():
    A, rows, cols, f = edge_problem(5)
    n = A.shape[0]
    rng = np.random.default_rng(0)
    w = Lr.init_weights(0)
    st = {}
    L0 = None
    for step in range(120):
        V = np.sign(rng.standard_normal((n, 8)))
        L, g, _ = Lr.kaporin_loss_grad(w, A, f, rows, cols, V)
        L0 = L if L0 is None else L0
        Lr.adam_step(w, g, st, lr=3e-3)
    assert L < L0
    o, _ = Lr.mlp_forward(w, f)
    G, _ = Lr.factor(o, rows, cols, A.diagonal(), n)
    bt = A @ np.random.default_rng(99).standard_normal((n, 3))
    for k in range(3):
        _, it_l = Lr.pcg(A, bt[:, k], lambda r: G.T @ (G @ r), tol=1e-8)
        _, it_j, _ = Fo.pcg(A, bt[:, k], tol=1e-8)
        assert it_l <= 0.7 * it_j, (it_l, it_j)


def _bad_weights():
    """Finite weights whose network makes G badly conditioned (outputs up to ~170)."""
    w = Lr.init_weights(4)
    rng = np.random.default_rng(14)
    w["W3"] = rng.normal(0, 20.0, w["W3"].shape)
    w["b1"] = rng.normal(0, 0.1, w["b1"].shape)
    return w


def test_stall_rule_and_fallback():
    """The fallback of the learned solve: a network giving Jacobi exactly never trips the stall
    rule (same iterations as plain Jacobi-PCG); finite but bad weights trip it (||r|| not 10 %
    lower over 10 iterations) long before the iteration cap, and Jacobi-PCG restarted from the
    iterate reaches the target; non-finite weights restart from the initial guess."""
    A, rows, cols, f = edge_problem(5)
    n = A.shape[0]
    b = A @ np.random.default_rng(7).standard_normal(n)
    _, it_j, _ = Fo.pcg(A, b, tol=1e-8)

    def apply_of(w):
        o, _ = Lr.mlp_forward(w, f)
        G, _ = Lr.factor(o, rows, cols, A.diagonal(), n)
        return lambda r: G.T @ (G @ r)

    x, il, ij, why = Lr.pcg_learned(A, b, apply_of(Lr.init_weights(0)), tol=1e-8, maxit=2000)
    assert why == "converged" and ij == 0 and abs(il - it_j) <= 1
    x, il, ij, why = Lr.pcg_learned(A, b, apply_of(_bad_weights()), tol=1e-8, maxit=2000)
    assert why == "stalled" and Lr.STALL_WINDOW <= il < 200
    assert np.linalg.norm(A @ x - b) <= 1.0001e-8 * np.linalg.norm(b)
    wn = Lr.init_weights(0)
    wn["b3"][0] = np.nan
    x, il, ij, why = Lr.pcg_learned(A, b, apply_of(wn), tol=1e-8, maxit=2000)
    assert why == "nonfinite" and il == 0 and abs(ij - it_j) <= 1
    assert np.linalg.norm(A @ x - b) <= 1.0001e-8 * np.linalg.norm(b)


def test_pair_energy_gradient_matches_finite_differences(small):
    A, rows, cols, f = small
    w = _random_weights(4)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((A.shape[0], 3))
    B = A @ X
    L, g = Lr.pair_energy_loss_grad(w, A, f, rows, cols, B, X)
    assert L > 0
    for _ in range(4):
        d = {k: rng.standard_normal(v.shape) for k, v in w.items()}
        h = 1e-7   # the loss is quartic in G: a smaller step keeps the third-order term below 1e-6
        Lp = Lr.pair_energy_loss_grad({k: w[k] + h * d[k] for k in w}, A, f, rows, cols, B, X)[0]
        Lm = Lr.pair_energy_loss_grad({k: w[k] - h * d[k] for k in w}, A, f, rows, cols, B, X)[0]
        fd = (Lp - Lm) / (2 * h)
        an = sum(np.sum(g[k] * d[k]) for k in w)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
    # the inverse Cholesky factor (full lower pattern) makes M = A^-1 exactly: the pairs' error vanishes
    G = np.linalg.inv(np.linalg.cholesky(A.toarray()))
    assert np.allclose(G.T @ G @ B, X, rtol=1e-8, atol=1e-10 * np.abs(X).max())


def solver_pairs(n_box, steps, seed):
    """(rhs, solution) pairs of the edge system from the oracle's own plasma cycle on an n^3 box
    at ten times the explicit limit: 10 electrons per tet, v_th = 1e6 m/s, uniform B_z = 0.1 T,
    density such that omega_p dt = 0.68 (as the 64^3 workload), a neutralising background; each
    step's rhs and the exact solution of A e* = rhs."""
    import scipy.sparse.linalg as sla
    from oracle.field import FieldOracle, init_fields
    from oracle.particles import ParticleOracle
    m = qi.BoxMesh(n_box)
    cx = Complex(m.xyz, m.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    po = ParticleOracle(cx, op.Minv)
    dt = 10 * 7.69e-10 / n_box
    fo = FieldOracle(cx, op, dt)
    dens = (0.68 / dt) ** 2 * qi.EPS0 * qi.ME / qi.QE ** 2
    npart = 10 * cx.Nt
    u_b, u_q = 2.0 ** -56, qi.QE * dens / npart * 2.0 ** -40
    x, v, tet = qi.uniform_plasma(m, npart, 1e6, seed=seed)
    e, b = init_fields(cx, qi.white(cx.Ne, seed, 3), qi.white(cx.Ne, seed, 5), 0.0, 0.1, 0.0, u_b)
    L = po.quantize_points(x.astype(np.float64), tet)
    Qbg = np.zeros(cx.Nn, np.int64)
    for i in range(4):
        np.add.at(Qbg, cx.tets[tet, i], -(1 << 20) * L[:, i])
    xo, vo, to = x.astype(np.float64), v.astype(np.float64), tet.astype(np.int64)
    Ac = fo.A.tocsc()
    R, Xs = [], []
    for _ in range(steps):
        out = po.push(e, b * u_b, xo, vo, to, -qi.QE / qi.ME, dt, -1)
        xo, vo, to = out["x"], out["v"], out["tet"]
        rhs = fo.rhs(e, b * u_b, out["g"] * u_q)
        R.append(rhs)
        Xs.append(sla.spsolve(Ac, rhs))
        e, b, _ = fo.step(e, b, u_b, out["g"], u_q, out["Q"], Qbg, tol=1e-12, tol_n=1e-12)
    return fo.A, np.array(R).T, np.array(Xs).T


@pytest.mark.slow
def test_training_on_solver_pairs():
    """Pairs of the plain solver (a 6^3 plasma cycle, seed 1; held out: seed 0) in the training
    objective. Measured here (iterations to 1e-8 on three held-out pairs): Jacobi 84-88,
    Kaporin number on Rademacher probes 33-34, the pairs' energy-norm loss alone 36-38,
    Kaporin + 0.5 x energy loss 33-34. Each learned variant beats Jacobi by more than half, and
    adding the pairs to the Kaporin objective costs nothing."""
    A, Btr, Xtr = solver_pairs(6, 60, 1)
    _, Bva, Xva = solver_pairs(6, 10, 0)
    n = A.shape[0]
    m = qi.BoxMesh(6)
    cx = Complex(m.xyz, m.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    ie = cx.int_edges
    tau = (10 * 7.69e-10 / 6) ** 2 / 4
    rows, cols = Lr.lower_pattern(A)
    ev = (cx.xyz[cx.edges[:, 1]] - cx.xyz[cx.edges[:, 0]])[ie]
    f = Lr.features(A, op.Meps[ie][:, ie].tocsr(), op.S[ie][:, ie].tocsr(), tau, ev, rows, cols)
    val = (3, 6, 9)
    it_j = [Fo.pcg(A, Bva[:, k], tol=1e-8)[1] for k in val]

    def train(kap, lam):
        w, st, r2 = Lr.init_weights(0), {}, np.random.default_rng(5)
        for _ in range(150):
            idx = r2.choice(Btr.shape[1], 8, replace=False)
            V = np.sign(r2.standard_normal((n, 8)))
            g = {k: 0.0 for k in w}
            if kap:
                _, gk, _ = Lr.kaporin_loss_grad(w, A, f, rows, cols, V)
                g = {k: g[k] + gk[k] for k in w}
            if lam:
                _, ge = Lr.pair_energy_loss_grad(w, A, f, rows, cols, Btr[:, idx], Xtr[:, idx])
                g = {k: g[k] + lam * ge[k] for k in w}
            Lr.adam_step(w, g, st, lr=3e-3)
        o, _ = Lr.mlp_forward(w, f)
        G, _ = Lr.factor(o, rows, cols, A.diagonal(), n)
        return [Lr.pcg(A, Bva[:, k], lambda r: G.T @ (G @ r), tol=1e-8, maxit=3000)[1] for k in val]

    it_k, it_e, it_ke = train(True, 0.0), train(False, 1.0), train(True, 0.5)
    for it in (it_k, it_e, it_ke):
        assert max(it) < 0.5 * min(it_j), (it, it_j)
    assert max(it_ke) <= max(it_k) + 2, (it_ke, it_k)


def _fsai(A):
    """Factorised sparse approximate inverse on the lower pattern of A: row i of G solves
    A[P_i, P_i] g = e_i over its pattern P_i (columns j <= i) and is scaled to g_i = sqrt(g_i);
    it minimises the Kaporin number of G A G^T over the pattern (Kolotilina and Yeremin)."""
    A = A.tocsr()
    n = A.shape[0]
    rows, cols, vals = [], [], []
    for i in range(n):
        P = np.sort(A.indices[A.indptr[i]:A.indptr[i + 1]])
        P = P[P <= i]
        sub = A[P][:, P].toarray()
        e = np.zeros(P.size)
        e[-1] = 1.0
        y = np.linalg.solve(sub, e)
        rows += [i] * P.size
        cols += list(P)
        vals += list(y / np.sqrt(y[-1]))
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


@pytest.mark.slow
def test_training_nears_the_best_factor_on_its_pattern():
    """The exact FSAI on the lower pattern of A (the best M = G^T G on that pattern for the
    Kaporin number) against the network trained by the oracle's own steps (Kaporin + 0.5 x the
    pairs' loss, 150 steps on a 6^3 plasma cycle's pairs): G A G^T of the FSAI has a unit diagonal
    (its normalisation) and the smallest Kaporin number among factors on the pattern, and the
    trained network needs at most 15 % more PCG iterations than it (measured: 34 against 32;
    Jacobi 86-88)."""
    A, Btr, Xtr = solver_pairs(6, 30, 1)
    _, Bva, _ = solver_pairs(6, 6, 0)
    n = A.shape[0]
    G = _fsai(A)
    GAG = (G @ A @ G.T).toarray()
    assert np.allclose(np.diag(GAG), 1.0, atol=1e-10)

    def kaporin(Gm):
        T = (Gm @ A @ Gm.T).toarray()
        return np.log(np.trace(T) / n) - np.linalg.slogdet(T)[1] / n

    # the FSAI beats random perturbations of itself on the pattern
    rng = np.random.default_rng(3)
    k0 = kaporin(G)
    for _ in range(3):
        Gp = G.copy()
        Gp.data = Gp.data * (1 + 0.05 * rng.standard_normal(Gp.data.size))
        assert kaporin(Gp) > k0
    it_fsai = [Lr.pcg(A, Bva[:, k], lambda r: G.T @ (G @ r), tol=1e-8)[1] for k in (2, 4)]
    m = qi.BoxMesh(6)
    cx = Complex(m.xyz, m.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    ie = cx.int_edges
    tau = (10 * 7.69e-10 / 6) ** 2 / 4
    rows, cols = Lr.lower_pattern(A)
    ev = (cx.xyz[cx.edges[:, 1]] - cx.xyz[cx.edges[:, 0]])[ie]
    f = Lr.features(A, op.Meps[ie][:, ie].tocsr(), op.S[ie][:, ie].tocsr(), tau, ev, rows, cols)
    w, st, r2 = Lr.init_weights(0), {}, np.random.default_rng(5)
    for _ in range(150):
        idx = r2.choice(Btr.shape[1], 8, replace=False)
        V = np.sign(r2.standard_normal((n, 8)))
        _, gk, _ = Lr.kaporin_loss_grad(w, A, f, rows, cols, V)
        _, ge = Lr.pair_energy_loss_grad(w, A, f, rows, cols, Btr[:, idx], Xtr[:, idx])
        Lr.adam_step(w, {k: gk[k] + 0.5 * ge[k] for k in w}, st, lr=3e-3)
    o, _ = Lr.mlp_forward(w, f)
    Gn, _ = Lr.factor(o, rows, cols, A.diagonal(), n)
    assert kaporin(Gn) > k0
    it_net = [Lr.pcg(A, Bva[:, k], lambda r: Gn.T @ (Gn @ r), tol=1e-8)[1] for k in (2, 4)]
    assert max(it_net) <= 1.15 * min(it_fsai), (it_net, it_fsai)
