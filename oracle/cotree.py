"""The literal quasi-Helmholtz reduced system (Sec. IV, dense, tiny meshes only).

Builds, on the interior edges and faces of a PEC box (Sec. IV.B):
  * an edge tree grounded on the PEC surface (all wall nodes merged into one root)
    and a face tree over the tets; the co-tree selectors C^e_c, C^b_c (eq. cotree_mat_e,
    eq. cotree_mat_b);
  * Sigma = [*eps][grad] (nodal potentials), Sigma_m = [div]^T (tet potentials, with
    the zero-mean constraint C_z^b of eq. zero_mean_constraint, alpha^3_i = 1);
  * the projectors P^Lambda_e = I - Sigma (G^T Sigma)^-1 G^T and
    P^Lambda_b = I - Sigma_m C_z (C_z^T D Sigma_m C_z)^-1 C_z^T D (eq. efld_mod_proj);
  * Z11..Z23 as printed in Sec. IV.B.2, and the trapezoidal (Newmark beta = 1/4,
    gamma = 1/2) march of eq. reduceMEs:
       Z11 (B^{n+1} - B^n) + dt/2 Z12 (E^{n+1} + E^n) = 0
       Z21 (E^{n+1} - E^n) - dt/2 Z22 (B^{n+1} + B^n) = -C_c^eT g - Z23 (E_ns^{n+1} - E_ns^n)
    with E_ns from the discrete Gauss law (eq. discreteGauss).
The Ampere line of eq. reduceMEs prints its current term without C_c^eT; the term
must be tested on the co-tree edges like the rest of the line, so it is read so.
Reconstruction: e = G E_ns + [*eps]^-1 P^Lambda_e [*eps] C^e_c E_s, b = P^Lambda_b C^b_c B_s.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from .complex_ import Complex
from .whitney import Operators


def edge_tree(cx: Complex, ie: np.ndarray, inn: np.ndarray, root_first=True, seed=None):
    """BFS spanning tree over interior nodes + one ground node; returns tree mask on ie."""
    gid = -np.ones(cx.Nn, dtype=np.int64)
    gid[inn] = np.arange(inn.size)
    ground = inn.size
    gid[cx.wall_node] = ground
    ends = gid[cx.edges[ie]]                      # (n_ie, 2) graph endpoints
    adj = [[] for _ in range(inn.size + 1)]
    order = np.arange(ie.size)
    if seed is not None:
        order = np.random.default_rng(seed).permutation(ie.size)
    for k in order:
        a, b = ends[k]
        if a != b:
            adj[a].append((b, k))
            adj[b].append((a, k))
    seen = np.zeros(inn.size + 1, bool)
    tree = np.zeros(ie.size, bool)
    start = ground if root_first else 0
    seen[start] = True
    dq = deque([start])
    while dq:
        u = dq.popleft()
        for w, k in adj[u]:
            if not seen[w]:
                seen[w] = True
                tree[k] = True
                dq.append(w)
    assert seen.all(), "interior graph not connected"
    return tree


def face_tree(cx: Complex, jf: np.ndarray, seed=None):
    """BFS spanning tree over tets through interior faces; returns tree mask on jf."""
    adj = [[] for _ in range(cx.Nt)]
    ft = {}
    for t in range(cx.Nt):
        for k in range(4):
            ft.setdefault(int(cx.tet_faces[t, k]), []).append(t)
    order = np.arange(jf.size)
    if seed is not None:
        order = np.random.default_rng(seed).permutation(jf.size)
    for k in order:
        a, b = ft[int(jf[k])]
        adj[a].append((b, k))
        adj[b].append((a, k))
    seen = np.zeros(cx.Nt, bool)
    tree = np.zeros(jf.size, bool)
    seen[0] = True
    dq = deque([0])
    while dq:
        u = dq.popleft()
        for w, k in adj[u]:
            if not seen[w]:
                seen[w] = True
                tree[k] = True
                dq.append(w)
    assert seen.all()
    return tree


class ReducedSystem:
    def __init__(self, cx: Complex, op: Operators, dt: float, tree_seed=None):
        self.cx, self.dt = cx, dt
        ie, inn = cx.int_edges, cx.int_nodes
        jf = np.flatnonzero(~cx.wall_face)
        self.ie, self.inn, self.jf = ie, inn, jf
        Me = op.Meps.toarray()[np.ix_(ie, ie)]
        Mm = op.Mmu.toarray()[np.ix_(jf, jf)]
        G = cx.G.toarray().astype(float)[np.ix_(ie, inn)]
        Cm = cx.C.toarray().astype(float)[np.ix_(jf, ie)]
        D = cx.D.toarray().astype(float)[:, jf]
        self.Me, self.Mm, self.G, self.Cm, self.D = Me, Mm, G, Cm, D
        n_t = cx.Nt
        Sigma = Me @ G
        PS_e = Sigma @ np.linalg.solve(G.T @ Sigma, G.T)
        self.PL_e = np.eye(ie.size) - PS_e
        Cz = np.zeros((n_t, n_t - 1))
        Cz[: n_t - 1] = np.eye(n_t - 1)
        Cz[n_t - 1] = -1.0                       # alpha^3_i = int W3_i = 1 for every tet
        Sm = D.T
        PS_b = Sm @ Cz @ np.linalg.solve(Cz.T @ D @ Sm @ Cz, Cz.T @ D)
        self.PL_b = np.eye(jf.size) - PS_b
        et = edge_tree(cx, ie, inn, seed=tree_seed)
        ftm = face_tree(cx, jf, seed=tree_seed)
        Ce = np.eye(ie.size)[:, ~et]
        Cb = np.eye(jf.size)[:, ~ftm]
        self.Ce, self.Cb = Ce, Cb
        Mei = np.linalg.inv(Me)
        self.Z11 = Cb.T @ self.PL_b @ Cb
        self.Z12 = Cb.T @ Cm @ Mei @ self.PL_e @ Me @ Ce
        self.Z13 = Cb.T @ Cm @ Mei @ Sigma
        self.Z21 = Ce.T @ self.PL_e @ Me @ Ce
        self.Z22 = Ce.T @ Cm.T @ Mm @ self.PL_b @ Cb
        self.Z23 = Ce.T @ Sigma
        self.K = G.T @ Sigma
        self.Mei = Mei
        h = 0.5 * dt
        nc = Ce.shape[1]
        self.lhs = np.block([[self.Z11, h * self.Z12], [-h * self.Z22, self.Z21]])
        self.rhs_m = np.block([[self.Z11, -h * self.Z12], [h * self.Z22, self.Z21]])
        self.nc = nc

    def decompose(self, e_int, b_int):
        """(E_ns, E_s, B_s) of interior edge values e and interior face fluxes b."""
        Ens = np.linalg.solve(self.K, self.G.T @ self.Me @ e_int)
        Es = np.linalg.lstsq(self.PL_e @ self.Me @ self.Ce, self.PL_e @ self.Me @ e_int, rcond=None)[0]
        Bs = np.linalg.lstsq(self.PL_b @ self.Cb, b_int, rcond=None)[0]
        return Ens, Es, Bs

    def compose(self, Ens, Es, Bs):
        e = self.G @ Ens + self.Mei @ self.PL_e @ self.Me @ self.Ce @ Es
        b = self.PL_b @ self.Cb @ Bs
        return e, b

    def step(self, Ens, Es, Bs, g_int, rho_new):
        """One trapezoidal step of eq. reduceMEs with E_ns^{n+1} from eq. discreteGauss."""
        Ens_new = np.linalg.solve(self.K, rho_new)
        rhs = self.rhs_m @ np.concatenate([Bs, Es])
        rhs[self.nc:] -= self.Ce.T @ g_int + self.Z23 @ (Ens_new - Ens)
        sol = np.linalg.solve(self.lhs, rhs)
        return Ens_new, sol[self.nc:], sol[: self.nc]
