"""Barycentric geometry, Whitney forms and the Hodge / mixed matrices (Sec. II.C).

  W0_i  = lambda_i
  W1_ab = lambda_a grad(lambda_b) - lambda_b grad(lambda_a)
  W2_abc = 2 (lambda_a grad(lambda_b) x grad(lambda_c) + lambda_b grad(lambda_c) x grad(lambda_a)
              + lambda_c grad(lambda_a) x grad(lambda_b))
  W3 = 1/|T|
Hodge matrices: [*eps]_ij = <W1_i, eps W1_j>, [*mu^-1]_ij = <W2_i, mu^-1 W2_j>,
[*rho]_ij = <W3_i, W3_j> (Sec. II.C). Mixed matrices M_g, M_c, M_d and the operators
[grad] = eps [*eps]^-1 M_g, [curl] = mu^-1 [*mu^-1]^-1 M_c, [div] = [*rho]^-1 M_d.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .complex_ import LOCAL_EDGES, LOCAL_FACES, Complex


def barycentric(cx: Complex):
    """Per tet: Minv (4x4) with lambda_i(r) = Minv[i,0] + Minv[i,1:] . r, and |T|."""
    P = cx.xyz[cx.tets]                       # (Nt, 4, 3)
    M = np.ones((cx.Nt, 4, 4))
    M[:, 1:, :] = P.transpose(0, 2, 1)        # columns are [1, x_i, y_i, z_i]
    Minv = np.linalg.inv(M)
    vol = np.abs(np.linalg.det(M)) / 6.0
    return Minv, vol


def lam_at(Minv_t: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Barycentric coordinates of points r (P,3) in tets Minv_t (P,4,4)."""
    return Minv_t[:, :, 0] + np.einsum("pij,pj->pi", Minv_t[:, :, 1:], r)


def w1_at(Minv_t, r, local_edge):
    a, b = local_edge
    lam = lam_at(Minv_t, r)
    g = Minv_t[:, :, 1:]
    return lam[:, a, None] * g[:, b] - lam[:, b, None] * g[:, a]


def w2_at(Minv_t, r, local_face):
    a, b, c = local_face
    lam = lam_at(Minv_t, r)
    g = Minv_t[:, :, 1:]
    return 2.0 * (lam[:, a, None] * np.cross(g[:, b], g[:, c])
                  + lam[:, b, None] * np.cross(g[:, c], g[:, a])
                  + lam[:, c, None] * np.cross(g[:, a], g[:, b]))


def field_E(cx: Complex, Minv, e: np.ndarray, tet: np.ndarray, r: np.ndarray) -> np.ndarray:
    """E(r) = sum_e e_e W1_e(r) over the six edges of the tet holding r."""
    Mt = Minv[tet]
    out = np.zeros_like(r)
    for k, le in enumerate(LOCAL_EDGES):
        out += e[cx.tet_edges[tet, k]][:, None] * w1_at(Mt, r, le)
    return out


def field_B(cx: Complex, Minv, b: np.ndarray, tet: np.ndarray, r: np.ndarray) -> np.ndarray:
    """B(r) = sum_f b_f W2_f(r) over the four faces of the tet holding r."""
    Mt = Minv[tet]
    out = np.zeros_like(r)
    for k, lf in enumerate(LOCAL_FACES):
        out += b[cx.tet_faces[tet, k]][:, None] * w2_at(Mt, r, lf)
    return out


# degree-2 exact 4-point rule on the reference tet (barycentric points, equal weights)
_A, _B = 0.5854101966249685, 0.1381966011250105
QUAD4 = np.array([[_A, _B, _B, _B], [_B, _A, _B, _B], [_B, _B, _A, _B], [_B, _B, _B, _A]])


def _assemble(rows_local, nrow_glob, ncol_glob, blocks, ridx, cidx):
    Nt = blocks.shape[0]
    r = np.repeat(ridx, cidx.shape[1], axis=1).reshape(Nt, ridx.shape[1], cidx.shape[1])
    c = np.repeat(cidx[:, None, :], ridx.shape[1], axis=1)
    return sp.csr_matrix((blocks.ravel(), (r.ravel(), c.ravel())), shape=(nrow_glob, ncol_glob))


def hodge_eps(cx: Complex, Minv, vol, eps: float):
    """[*eps] = eps <W1_i, W1_j> in closed form with int lambda_i lambda_j = |T|(1+d_ij)/20."""
    g = Minv[:, :, 1:]
    GG = np.einsum("tik,tjk->tij", g, g)      # grad lambda_i . grad lambda_j
    Lm = (np.ones((4, 4)) + np.eye(4)) / 20.0
    blk = np.zeros((cx.Nt, 6, 6))
    for p, (a, b) in enumerate(LOCAL_EDGES):
        for q, (c, d) in enumerate(LOCAL_EDGES):
            blk[:, p, q] = (Lm[a, c] * GG[:, b, d] - Lm[a, d] * GG[:, b, c]
                            - Lm[b, c] * GG[:, a, d] + Lm[b, d] * GG[:, a, c])
    blk *= (eps * vol)[:, None, None]
    return _assemble(None, cx.Ne, cx.Ne, blk, cx.tet_edges, cx.tet_edges)


def hodge_muinv(cx: Complex, Minv, vol, mu: float):
    """[*mu^-1] = mu^-1 <W2_i, W2_j>, integrated with the degree-2 exact 4-point rule."""
    Nt = cx.Nt
    P = cx.xyz[cx.tets]
    blk = np.zeros((Nt, 4, 4))
    for qp in QUAD4:
        r = np.einsum("i,tid->td", qp, P)
        W = np.stack([w2_at(Minv, r, lf) for lf in LOCAL_FACES], axis=1)  # (Nt,4,3)
        blk += 0.25 * np.einsum("tik,tjk->tij", W, W)
    blk *= (vol / mu)[:, None, None]
    return _assemble(None, cx.Nf, cx.Nf, blk, cx.tet_faces, cx.tet_faces)


def hodge_rho(cx: Complex, vol):
    """[*rho] = <W3_i, W3_j> = diag(1/|T|)."""
    return sp.diags(1.0 / vol)


def mixed_g(cx: Complex, Minv, vol):
    """M_g[e, n] = <W1_e, grad W0_n> (closed form, int lambda_i = |T|/4)."""
    g = Minv[:, :, 1:]
    GG = np.einsum("tik,tjk->tij", g, g)
    blk = np.zeros((cx.Nt, 6, 4))
    for p, (a, b) in enumerate(LOCAL_EDGES):
        for n in range(4):
            blk[:, p, n] = 0.25 * (GG[:, b, n] - GG[:, a, n])
    blk *= vol[:, None, None]
    return _assemble(None, cx.Ne, cx.Nn, blk, cx.tet_edges, cx.tets)


def mixed_c(cx: Complex, Minv, vol):
    """M_c[f, e] = <W2_f, curl W1_e>; curl W1_ab = 2 grad(lambda_a) x grad(lambda_b)."""
    Nt = cx.Nt
    P = cx.xyz[cx.tets]
    g = Minv[:, :, 1:]
    curls = np.stack([2.0 * np.cross(g[:, a], g[:, b]) for a, b in LOCAL_EDGES], axis=1)
    blk = np.zeros((Nt, 4, 6))
    for qp in QUAD4:
        r = np.einsum("i,tid->td", qp, P)
        W = np.stack([w2_at(Minv, r, lf) for lf in LOCAL_FACES], axis=1)
        blk += 0.25 * np.einsum("tik,tjk->tij", W, curls)
    blk *= vol[:, None, None]
    return _assemble(None, cx.Nf, cx.Ne, blk, cx.tet_faces, cx.tet_edges)


def mixed_d(cx: Complex, Minv, vol):
    """M_d[t, f] = <W3_t, div W2_f>; div W2_abc = 6 grad(la) . (grad(lb) x grad(lc))."""
    g = Minv[:, :, 1:]
    blk = np.zeros((cx.Nt, 1, 4))
    for k, (a, b, c) in enumerate(LOCAL_FACES):
        div = 6.0 * np.einsum("ti,ti->t", g[:, a], np.cross(g[:, b], g[:, c]))
        blk[:, 0, k] = div  # integral of (1/|T|) * div over |T|
    return _assemble(None, cx.Nt, cx.Nf, blk, np.arange(cx.Nt)[:, None], cx.tet_faces)


class Operators:
    """All matrices of the semi-discrete system on one mesh."""

    def __init__(self, cx: Complex, eps: float, mu: float):
        self.cx = cx
        self.eps, self.mu = eps, mu
        self.Minv, self.vol = barycentric(cx)
        self.Meps = hodge_eps(cx, self.Minv, self.vol, eps).tocsr()
        self.Mmu = hodge_muinv(cx, self.Minv, self.vol, mu).tocsr()
        C = cx.C.astype(np.float64)
        G = cx.G.astype(np.float64)
        self.S = (C.T @ self.Mmu @ C).tocsr()          # [*S] = [curl]^T [*mu^-1] [curl]
        self.K = (G.T @ self.Meps @ G).tocsr()         # discrete Laplacian G^T [*eps] G
        self.CtMmu = (C.T @ self.Mmu).tocsr()

    def stiffness_p1(self):
        """eps * sum_T |T| grad(lambda_i) . grad(lambda_j): the P1 stiffness matrix."""
        g = self.Minv[:, :, 1:]
        blk = self.eps * self.vol[:, None, None] * np.einsum("tik,tjk->tij", g, g)
        return _assemble(None, self.cx.Nn, self.cx.Nn, blk, self.cx.tets, self.cx.tets)

    def curlcurl_nedelec(self):
        """mu^-1 sum_T |T| curl W1_i . curl W1_j with curl W1_ab = 2 grad(la) x grad(lb)."""
        g = self.Minv[:, :, 1:]
        curls = np.stack([2.0 * np.cross(g[:, a], g[:, b]) for a, b in LOCAL_EDGES], axis=1)
        blk = (self.vol / self.mu)[:, None, None] * np.einsum("tik,tjk->tij", curls, curls)
        return _assemble(None, self.cx.Ne, self.cx.Ne, blk, self.cx.tet_edges, self.cx.tet_edges)
