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
            self.Kz = (self.Cz.T @ self.K @ self.Cz).tocsr()
            self.alpha = alpha
        self.Gf = cx.G.astype(np.float64).tocsr()
        self.GtMeps = (self.Gf.T @ op.Meps).tocsr()
        self.Gint = self.Gf[:, inn].tocsr()

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

    def step(self, e, b_int, u_b, g_int, u_q, Q_new, Q_bg, tol=1e-12, tol_n=1e-12, gauss=True):
        """One field update with rho^{n+1} = u_q (Q_bg - Q^{n+1}) on the interior nodes."""
        rho = u_q * (Q_bg - Q_new).astype(np.float64)[self.inn]
        return self.step_with_rho(e, b_int, u_b, g_int, u_q, rho, tol, tol_n, gauss)

    def step_with_rho(self, e, b_int, u_b, g_int, u_q, rho, tol=1e-12, tol_n=1e-12, gauss=True):
        """One field update given rho^{n+1} on the interior nodes. Returns (e, b, info)."""
        b_real = b_int.astype(np.float64) * u_b
        rhs = self.rhs(e, b_real, g_int.astype(np.float64) * u_q)
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

    def wave_step(self, e, e_prev, b_int, u_b, g_int, g_prev_int, u_q, rho, tol=1e-12, tol_n=1e-12, gauss=True):
        """One wave-equation update given e^n, e^{n-1}, the step currents g^{n+1/2}, g^{n-1/2}
        and rho^{n+1} on the interior nodes. Returns (e^{n+1}, b^{n+1}, info)."""
        rhs = self.wave_rhs(e, e_prev, (g_int - g_prev_int).astype(np.float64) * u_q)
        xs, it, res = pcg(self.A, rhs, x0=e[self.ie].copy(), tol=tol)
        es = np.zeros_like(e)
        es[self.ie] = xs
        info = dict(edge_it=it, edge_res=res)
        e_new = self.gauss_project(es, rho, tol_n, info) if gauss else es
        info["gauss_res"] = self.gauss_error(e_new, rho)
        u = np.rint(0.5 * self.dt * (e_new + e) / u_b).astype(np.int64)
        return e_new, b_int - self.cx.C @ u, info


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
