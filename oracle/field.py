"""Implicit field update of the quasi-Helmholtz PIC cycle, FP64 (test infrastructure).

Semi-discrete system (Sec. II.C, eq. maxwell_semi), with [curl] = C (face x edge
incidence) once B is carried by face fluxes and E by edge DOFs:
    d/dt b + C e = 0,        [*eps] d/dt e - C^T [*mu^-1] b = -J
Time discretisation: Newmark beta = 1/4, gamma = 1/2 (Sec. IV.B.2 names Newmark-beta and
defers constants to another paper; this pair is the trapezoidal rule). Eliminating
b^{n+1} gives one SPD system on the interior edges,
    ([*eps] + tau S) e* = ([*eps] - tau S) e^n + dt C^T [*mu^-1] b^n - g,   tau = dt^2/4,
with g the current integrated over the step (the path integral of Sec. IV.B.1).
The non-solenoidal part is then fixed by the discrete Gauss law (eq. discreteGauss):
    G^T [*eps] G delta = rho^{n+1} - G^T [*eps] e*,    e^{n+1} = e* + G delta,
so that G^T [*eps] e^{n+1} = rho^{n+1} to the solver tolerance; rho = -u_q Q + rho_bg
with Q the Whitney-0 charge (sign: Gauss's law tested with W0 gives -G^T D = Q).
Faraday's law updates integer face fluxes, b^{n+1} = b^n - C u with
u = round((dt/2)(e^{n+1} + e^n) / u_b), so [div] b = D b never changes (D C = 0;
Sec. IV.A: B_ns = 0 makes the magnetic Gauss law hold by construction).
This equals the literal tree/co-tree system (cotree.py) in exact arithmetic.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .complex_ import Complex
from .whitney import Operators


def pcg(A, b, x0=None, tol=1e-12, maxit=10000, diag=None):
    """Jacobi-preconditioned CG (Hestenes-Stiefel), stop at ||b - A x|| <= tol ||b||."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    d = A.diagonal() if diag is None else diag
    r = b - A @ x
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    z = r / d
    p = z.copy()
    rz = r @ z
    it = 0
    res = np.linalg.norm(r) / nb
    while res > tol and it < maxit:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = r / d
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        res = np.linalg.norm(r) / nb
    return x, it, res


class FieldOracle:
    def __init__(self, cx: Complex, op: Operators, dt: float):
        self.cx, self.op, self.dt = cx, op, dt
        self.tau = dt * dt / 4.0
        ie, inn = cx.int_edges, cx.int_nodes
        self.ie, self.inn = ie, inn
        A = (op.Meps + self.tau * op.S).tocsr()
        self.A = A[ie][:, ie].tocsr()
        self.Bm = (op.Meps - self.tau * op.S).tocsr()
        self.K = op.K[inn][:, inn].tocsr()
        if cx.neumann:
            # natural boundary: K has the constants as null space; the potential is fixed by the
            # zero-mean constraint of eq. zero_mean_constraint, delta = C_z y with the last
            # node's value -sum_i alpha_i y_i / alpha_n, alpha_i = integral of W0_i
            P = cx.xyz[cx.tets]
            vol = np.abs(np.einsum("ti,ti->t", P[:, 1] - P[:, 0], np.cross(P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]))) / 6.0
            alpha = np.bincount(cx.tets.ravel(), weights=np.repeat(vol / 4.0, 4), minlength=cx.Nn)
            n = cx.Nn
            top = sp.identity(n - 1, format="csr")
            last = sp.csr_matrix(-alpha[:-1] / alpha[-1])
            self.Cz = sp.vstack([top, last]).tocsr()
            self.alpha = alpha
            self._Kz = None
        self.Gf = cx.G.astype(np.float64).tocsr()
        self.GtMeps = (self.Gf.T @ op.Meps).tocsr()
        self.Gint = self.Gf[:, inn].tocsr()

    @property
    def Kz(self):
        """C_z^T K C_z (formed at first use: its last row and column are dense)."""
        if self._Kz is None:
            self._Kz = (self.Cz.T @ self.K @ self.Cz).tocsr()
        return self._Kz

    def decompose(self, e, tol=1e-13):
        """Quasi-Helmholtz split of the edge field (Sec. III: the projector P^Sigma_e with the
        zero-mean constraint of eq. zero_mean_constraint): rho_bar = G^T [*eps] e on the
        unknown nodes, E_ns = K^{-1} rho_bar (node coefficients of the potential part; zero on
        PEC walls, zero W0-weighted mean under natural walls), E_s = e - G E_ns (edge
        coefficients, G^T [*eps] E_s = 0). Returns (E_ns on all nodes, E_s on all edges,
        rho_bar on the unknown nodes)."""
        rho_bar = (self.GtMeps @ e)[self.inn]
        if self.cx.neumann:
            y, _, _ = pcg(self.Kz, self.Cz.T @ rho_bar, tol=tol)
            phi = self.Cz @ y
        else:
            phi, _, _ = pcg(self.K, rho_bar, tol=tol)
        e_ns = np.zeros(self.cx.Nn)
        e_ns[self.inn] = phi
        return e_ns, e - self.Gint @ phi, rho_bar

    def rhs(self, e, b_real, g_real):
        r = self.Bm @ e + self.dt * (self.op.CtMmu @ b_real) - g_real
        return r[self.ie]

    def gauss_residual(self, e, rho):
        return rho - (self.GtMeps @ e)[self.inn]

    def gauss_scale(self, e, rho):
        """||rho|| + || |G^T [*eps]| |e| ||: the size of the terms that cancel in the
        discrete Gauss law (normwise backward-error scaling of its residual)."""
        absop = abs(self.GtMeps[self.inn])
        return np.linalg.norm(rho) + np.linalg.norm(absop @ np.abs(e))

    def gauss_error(self, e, rho):
        return np.linalg.norm(self.gauss_residual(e, rho)) / self.gauss_scale(e, rho)

    def gauss_project(self, es, rho, tol_n, info):
        """e = e* + G delta with G^T [*eps] G delta = rho - G^T [*eps] e* (eq. discreteGauss),
        solved until the Gauss residual is below tol_n times its scale."""
        rg = self.gauss_residual(es, rho)
        scale = self.gauss_scale(es, rho)
        if scale > 0 and np.linalg.norm(rg) > tol_n * scale:
            tol_rel = tol_n * scale / np.linalg.norm(rg)
            if self.cx.neumann:
                rz = self.Cz.T @ rg
                y, itn, _ = pcg(self.Kz, rz, tol=tol_rel * np.linalg.norm(rg) / max(np.linalg.norm(rz), 1e-300))
                dl = self.Cz @ y
            else:
                dl, itn, _ = pcg(self.K, rg, tol=tol_rel)
        else:
            dl, itn = np.zeros(self.inn.size), 0
        info.update(node_it=itn)
        return es + self.Gint @ dl

    def step(self, e, b_int, u_b, g_int, u_q, Q_new, Q_bg, tol=1e-12, tol_n=1e-12, gauss=True, h_sum=None):
        """One field update with rho^{n+1} = u_q (Q_bg - Q^{n+1}) on the interior nodes."""
        rho = u_q * (Q_bg - Q_new).astype(np.float64)[self.inn]
        return self.step_with_rho(e, b_int, u_b, g_int, u_q, rho, tol, tol_n, gauss, h_sum)

    def step_with_rho(self, e, b_int, u_b, g_int, u_q, rho, tol=1e-12, tol_n=1e-12, gauss=True, h_sum=None):
        """One field update given rho^{n+1} on the interior nodes; h_sum: the boundary source
        dt/2 (h^n + h^{n+1}) on every edge, or None. Returns (e, b, info)."""
        b_real = b_int.astype(np.float64) * u_b
        rhs = self.rhs(e, b_real, g_int.astype(np.float64) * u_q)
        if h_sum is not None:
            rhs = rhs + h_sum[self.ie]
        x0 = e[self.ie].copy()
        xs, it, res = pcg(self.A, rhs, x0=x0, tol=tol)
        es = np.zeros_like(e)
        es[self.ie] = xs
        info = dict(edge_it=it, edge_res=res)
        e_new = self.gauss_project(es, rho, tol_n, info) if gauss else es
        info["gauss_res"] = self.gauss_error(e_new, rho)
        u = np.rint(0.5 * self.dt * (e_new + e) / u_b).astype(np.int64)
        b_new = b_int - self.cx.C @ u
        return e_new, b_new, info


class WaveOracle(FieldOracle):
    """Edge update of the wave equation (eq. wave_cont): [*eps] e'' + S e = -J', S = C^T [*mu^-1] C,
    with Newmark beta = 1/4, gamma = 1/2 (the constants of the trapezoidal rule, reading R1):
        ([*eps] + tau S) e^{n+1} = [*eps](2 e^n - e^{n-1}) - tau S (2 e^n + e^{n-1})
                                   - (g^{n+1/2} - g^{n-1/2}),
    the forcing dt^2 J' taken as the difference of the currents integrated over the two steps
    around t^n (the path integrals of Sec. IV.B.1). G^T S = 0 then gives G^T [*eps] of the second
    difference of e equal to the second difference of the charge: the discrete Gauss law is
    kept up to what each solve leaves in the irrotational part, and that error grows linearly
    in time (the t grad Phi null space, Sec. V) unless the Gauss-law correction removes it.
    Face fluxes follow Faraday's law in integers as in FieldOracle."""

    def wave_rhs(self, e, e_prev, dg_real):
        r = self.op.Meps @ (2.0 * e - e_prev) - self.tau * (self.op.S @ (2.0 * e + e_prev)) - dg_real
        return r[self.ie]

    def wave_step(self, e, e_prev, b_int, u_b, g_int, g_prev_int, u_q, rho, tol=1e-12, tol_n=1e-12, gauss=True,
                  h_diff=None):
        """One wave-equation update given e^n, e^{n-1}, the step currents g^{n+1/2}, g^{n-1/2}
        and rho^{n+1} on the interior nodes; h_diff: the boundary source dt/2 (h^{n+1} - h^{n-1})
        on every edge, or None. Returns (e^{n+1}, b^{n+1}, info)."""
        rhs = self.wave_rhs(e, e_prev, (g_int - g_prev_int).astype(np.float64) * u_q)
        if h_diff is not None:
            rhs = rhs + h_diff[self.ie]
        xs, it, res = pcg(self.A, rhs, x0=e[self.ie].copy(), tol=tol)
        es = np.zeros_like(e)
        es[self.ie] = xs
        info = dict(edge_it=it, edge_res=res)
        e_new = self.gauss_project(es, rho, tol_n, info) if gauss else es
        info["gauss_res"] = self.gauss_error(e_new, rho)
        u = np.rint(0.5 * self.dt * (e_new + e) / u_b).astype(np.int64)
        return e_new, b_int - self.cx.C @ u, info


# Dunavant's degree-4 rule on a triangle: barycentric points and weights (summing to 1)
_DUNAVANT4 = [((0.108103018168070, 0.445948490915965, 0.445948490915965), 0.223381589678011),
              ((0.445948490915965, 0.108103018168070, 0.445948490915965), 0.223381589678011),
              ((0.445948490915965, 0.445948490915965, 0.108103018168070), 0.223381589678011),
              ((0.816847572980459, 0.091576213509771, 0.091576213509771), 0.109951743655322),
              ((0.091576213509771, 0.816847572980459, 0.091576213509771), 0.109951743655322),
              ((0.091576213509771, 0.091576213509771, 0.816847572980459), 0.109951743655322)]


class PlaneWave:
    """Plane wave entering through a natural boundary (the Neumann test of Sec. VI.A.2): E along
    -z, travelling along +x, with the time signature of a derivative of a modulated Gaussian (our
    own; the paper's formula is in a reference that is not available),
        s(u) = exp(-u^2 / (2 sig^2)) cos(2 pi f0 u), u = tau - t0, sig = 1 / (2 pi bw),
        E_inc = -z E0 s'(t - x/c),   H_inc = y (E0 / eta) s'(t - x/c).
    Integrating W1_i . curl H by parts in Ampere's law leaves the boundary term
    h_i(t) = integral over the boundary of W1_i . (n x H_inc) dS (n outward), taken here with
    Dunavant's degree-4 rule on every boundary face; the trapezoidal update adds
    dt/2 (h^n + h^{n+1}) to its right-hand side, the wave update dt/2 (h^{n+1} - h^{n-1})."""

    def __init__(self, cx: Complex, op: Operators, E0, f0, bw, t0, faces=None):
        """faces: the wall faces to integrate over (all by default); h is then complete on the
        edges all of whose wall faces are listed."""
        from .whitney import w1_at
        from .complex_ import LOCAL_EDGES, LOCAL_FACES
        self.cx, self.E0, self.f0, self.t0 = cx, E0, f0, t0
        self.sig = 1.0 / (2.0 * np.pi * bw)
        eps, mu = op.eps, op.mu
        self.c = 1.0 / np.sqrt(eps * mu)
        self.eta = np.sqrt(mu / eps)
        # per boundary face and rule point: x of the point and, for the face's three edges, the
        # weight times W1_i . (n x y-hat)
        edges, coef, xq = [], [], []
        slot = np.flatnonzero(cx.wall_face[cx.tet_faces.ravel()])   # a wall face has one tet
        if faces is not None:
            slot = slot[np.isin(cx.tet_faces.ravel()[slot], faces)]
        for t, k in zip(*np.divmod(slot, 4)):
            verts = LOCAL_FACES[k]
            P = cx.xyz[cx.tets[t, list(verts)]]
            area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
            gk = op.Minv[t, k, 1:]
            nvec = -gk / np.linalg.norm(gk)               # outward: lambda_k grows inward
            nxy = np.cross(nvec, np.array([0.0, 1.0, 0.0]))
            on_face = [j for j, (a, b) in enumerate(LOCAL_EDGES) if a in verts and b in verts]
            for bary, w in _DUNAVANT4:
                r = bary[0] * P[0] + bary[1] * P[1] + bary[2] * P[2]
                for j in on_face:
                    W = w1_at(op.Minv[t][None], r[None], LOCAL_EDGES[j])[0]
                    edges.append(cx.tet_edges[t, j])
                    coef.append(w * area * (W @ nxy))
                    xq.append(r[0])
        self.edges, self.coef, self.xq = np.array(edges), np.array(coef), np.array(xq)

    def ds(self, tau):
        """s'(tau)."""
        u = tau - self.t0
        om = 2.0 * np.pi * self.f0
        env = np.exp(-u * u / (2.0 * self.sig ** 2))
        return env * (-(u / self.sig ** 2) * np.cos(om * u) - om * np.sin(om * u))

    def h(self, t):
        """Boundary term h(t) on every edge (zero off the boundary)."""
        out = np.zeros(self.cx.Ne)
        np.add.at(out, self.edges, self.coef * (self.E0 / self.eta) * self.ds(t - self.xq / self.c))
        return out

    def e_line(self, t, npts=5):
        """Line integrals of E_inc along every edge at time t (Gauss-Legendre)."""
        xg, wg = np.polynomial.legendre.leggauss(npts)
        a, b = self.cx.xyz[self.cx.edges[:, 0]], self.cx.xyz[self.cx.edges[:, 1]]
        out = np.zeros(self.cx.Ne)
        for s_, w in zip(0.5 * (xg + 1.0), 0.5 * wg):
            x = a[:, 0] + s_ * (b[:, 0] - a[:, 0])
            out += w * (-self.E0 * self.ds(t - x / self.c)) * (b[:, 2] - a[:, 2])
        return out


def init_fields(cx: Complex, white_e, white_a, sigma_e, bz, sigma_b, u_b):
    """Synthetic initial fields.

    e_e = l_e sigma_e w_e on interior edges (0 on PEC walls);
    a_e = line integral of A = (0, bz x, 0) along the edge + sigma_b l_e^2/(2 sqrt 3) w'_e,
    a_int = round(a / u_b), b = C a_int (int64), so that D b = 0 exactly and the flux
    density is uniform bz z-hat plus a random curl with face-flux spread ~ sigma_b |f|.
    """
    ell = cx.edge_lengths()
    e = ell * sigma_e * white_e
    if not cx.neumann:
        e[cx.wall_edge] = 0.0
    xa, xb = cx.xyz[cx.edges[:, 0]], cx.xyz[cx.edges[:, 1]]
    a = bz * 0.5 * (xa[:, 0] + xb[:, 0]) * (xb[:, 1] - xa[:, 1])
    a = a + sigma_b * ell ** 2 / (2.0 * np.sqrt(3.0)) * white_a
    a_int = np.rint(a / u_b).astype(np.int64)
    b = cx.C @ a_int
    return e, b


def dt_cfl(op: Operators, cx: Complex, tol=1e-8) -> float:
    """Leap-frog stability limit 2/sqrt(lambda_max([*eps]^-1 S)) on the interior edges."""
    import scipy.sparse.linalg as sla
    ie = cx.int_edges
    M = op.Meps[ie][:, ie].tocsc()
    S = op.S[ie][:, ie].tocsc()
    lu = sla.splu(M)
    Op = sla.LinearOperator(M.shape, matvec=lambda x: lu.solve(S @ x), dtype=np.float64)
    lam = sla.eigs(Op, k=1, which="LM", tol=tol, return_eigenvectors=False)
    return 2.0 / np.sqrt(abs(lam[0].real))
