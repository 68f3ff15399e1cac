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
