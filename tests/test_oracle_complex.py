"""Pins of the oracle's mesh complex and Whitney operators (Sec. II.C, Sec. IV.B, Sec. V).

Each test checks the oracle against something other than itself: integer identities of
the de Rham complex, closed-form counts of the Kuhn lattice, Euler's relation, and the
paper's statements that [grad], [curl], [div] built from Hodge and mixed matrices are the
incidence matrices, that G^T [*eps] G is the discrete Laplacian, and that the co-tree
edge and face counts agree on a simply connected domain (Sec. V, item 7).
"""
import numpy as np
import pytest

import qh_inputs as qi
from oracle.complex_ import Complex
from oracle import whitney as W


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_kuhn_counts_closed_form(n):
    m = qi.BoxMesh(n)
    cx = Complex(m.xyz, m.tets)
    assert cx.Nn == (n + 1) ** 3
    assert cx.Nt == 6 * n ** 3
    assert cx.Ne == 3 * n * (n + 1) ** 2 + 3 * n ** 2 * (n + 1) + n ** 3
    assert cx.Nf == 12 * n ** 3 + 6 * n ** 2
    assert cx.wall_face.sum() == 12 * n ** 2
    assert cx.wall_edge.sum() == 18 * n ** 2
    assert cx.wall_node.sum() == (n + 1) ** 3 - max(n - 1, 0) ** 3


def test_complex_identities(jitter4):
    _, cx, _ = jitter4
    assert abs(cx.C @ cx.G).max() == 0          # curl grad = 0
    assert abs(cx.D @ cx.C).max() == 0          # div curl = 0
    assert cx.Nn - cx.Ne + cx.Nf - cx.Nt == 1   # Euler characteristic of a ball
    # every interior face has two tets, every wall face one
    assert set(np.unique(cx.face_count)) == {1, 2}


def test_cotree_counts_equal(jitter4):
    """#E_s = #B_s for a simply connected PEC box (Sec. V item 7)."""
    _, cx, _ = jitter4
    n_cotree_edges = cx.int_edges.size - cx.int_nodes.size
    n_cotree_faces = int((~cx.wall_face).sum()) - (cx.Nt - 1)
    assert n_cotree_edges == n_cotree_faces == 289


def test_operators_are_incidence(jitter4):
    """[grad] = eps [*eps]^-1 M_g = G, [curl] = mu^-1 [*mu^-1]^-1 M_c = C, [div] = D."""
    _, cx, op = jitter4
    Mg = W.mixed_g(cx, op.Minv, op.vol).toarray()
    grad = qi.EPS0 * np.linalg.solve(op.Meps.toarray(), Mg)
    assert np.allclose(grad, cx.G.toarray(), atol=1e-12)
    Mc = W.mixed_c(cx, op.Minv, op.vol).toarray()
    curl = np.linalg.solve(op.Mmu.toarray(), Mc) / qi.MU0
    assert np.allclose(curl, cx.C.toarray(), atol=1e-12)
    Md = W.mixed_d(cx, op.Minv, op.vol).toarray()
    div = np.linalg.solve(W.hodge_rho(cx, op.vol).toarray(), Md)
    assert np.allclose(div, cx.D.toarray(), atol=1e-12)


def test_laplacian_and_curlcurl_two_formulas(jitter4):
    """G^T [*eps] G equals the P1 stiffness matrix; C^T [*mu^-1] C the Nedelec curl-curl."""
    _, _, op = jitter4
    K1, K2 = op.K.toarray(), op.stiffness_p1().toarray()
    assert np.abs(K1 - K2).max() <= 1e-13 * np.abs(K2).max()
    S1, S2 = op.S.toarray(), op.curlcurl_nedelec().toarray()
    assert np.abs(S1 - S2).max() <= 1e-13 * np.abs(S2).max()


def test_hodge_matrices_spd(jitter4):
    _, _, op = jitter4
    for M in (op.Meps, op.Mmu):
        A = M.toarray()
        assert np.allclose(A, A.T, rtol=0, atol=1e-14 * np.abs(A).max())
        assert np.linalg.eigvalsh(A).min() > 0


def test_whitney_reproduces_constants(jitter4):
    """Edge DOFs of a uniform E and face fluxes of a uniform B are reproduced exactly."""
    _, cx, op = jitter4
    rng = np.random.default_rng(7)
    E0 = np.array([1.5, -0.25, 0.75])
    B0 = np.array([-0.3, 0.1, 0.2])
    x = cx.xyz
    e = (x[cx.edges[:, 1]] - x[cx.edges[:, 0]]) @ E0
    fa, fb, fc = (x[cx.faces[:, k]] for k in range(3))
    b = 0.5 * np.cross(fb - fa, fc - fa) @ B0
    tet = rng.integers(0, cx.Nt, 200)
    w = rng.dirichlet(np.ones(4), 200)
    r = np.einsum("pi,pid->pd", w, x[cx.tets[tet]])
    assert np.allclose(W.field_E(cx, op.Minv, e, tet, r), E0, atol=1e-12)
    assert np.allclose(W.field_B(cx, op.Minv, b, tet, r), B0, atol=1e-12)


def test_tangential_and_normal_continuity(jitter4):
    """W1 fields have continuous tangential E, W2 fields continuous normal B across faces."""
    _, cx, op = jitter4
    rng = np.random.default_rng(3)
    e = rng.standard_normal(cx.Ne)
    b = rng.standard_normal(cx.Nf)
    inner = np.flatnonzero(cx.face_count == 2)[:50]
    for f in inner:
        tt = [t for t in range(cx.Nt) if f in cx.tet_faces[t]]
        P = cx.xyz[cx.faces[f]]
        w = rng.dirichlet(np.ones(3))
        r = (w @ P)[None, :]
        n = np.cross(P[1] - P[0], P[2] - P[0])
        E = [W.field_E(cx, op.Minv, e, np.array([t]), r)[0] for t in tt]
        B = [W.field_B(cx, op.Minv, b, np.array([t]), r)[0] for t in tt]
        assert np.allclose(np.cross(E[0], n), np.cross(E[1], n), atol=1e-10)
        assert np.isclose(B[0] @ n, B[1] @ n, atol=1e-10)
