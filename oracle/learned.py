"""FP64 oracle of the learned preconditioner for the edge system (test infrastructure).

The edge system A e = rhs (A = [*eps] + dt^2/4 S on the interior edges) is solved by
preconditioned CG with either the Jacobi preconditioner or a learned one. The learned
preconditioner is M = G^T G with G sparse and lower triangular on the pattern of A, so M is
symmetric positive definite whenever the diagonal of G is positive. A small network maps 16
local features of each pattern entry (i, j), j <= i, to o_ij and
    G_ij = o_ij / sqrt(A_jj)  (j < i),    G_ii = softplus(o_ii + s0) / sqrt(A_ii),
with softplus(s0) = 1, so a network that outputs 0 gives G = D^-1/2 and M = D^-1 (Jacobi).
Network: 16 -> 64 -> 64 -> 1, ReLU.

Training objective: the Kaporin condition number of G A G^T,
    K = (tr(G A G^T) / n) / det(G A G^T)^(1/n),
whose logarithm is, for triangular G and up to the constant log det A / n,
    L = log(tr(G A G^T) / n) - (2/n) sum_i log G_ii,
with tr(G A G^T)/n estimated by T = mean_p v_p^T G A G^T v_p / |v_p|^2 over Rademacher probes.
K >= 1 with equality iff G A G^T is a multiple of I; CG converges in a number of iterations
bounded through K, and L does not depend on the scale of G. Gradient (w_p = G^T v_p):
    dL/dG_ij = (2 / (P T)) sum_p (A w_p)_j v_p,i / |v_p|^2  - [i = j] 2 / (n G_ii).
Solver pairs (b, x) with A x = b, from the plain solver, enter training through the energy-norm
loss L_E = mean ||x - M b||_A^2 / ||x||_A^2 (pair_energy_loss_grad), added to L with a weight;
they also measure the result: PCG iterations to 1e-8 and the energy-norm error.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

F_IN, HID = 16, 64


def lower_pattern(A: sp.csr_matrix):
    """Rows, cols of the lower triangle (j <= i) of A's pattern, row-major, sorted."""
    C = sp.tril(A, format="coo")
    order = np.lexsort((C.col, C.row))
    return C.row[order].astype(np.int64), C.col[order].astype(np.int64)


def features(A, Meps, S, tau, edge_vec, rows, cols):
    """16 dimensionless features per lower-pattern entry (i, j)."""
    A = A.tocsr()
    dA = A.diagonal()
    dM = Meps.diagonal()
    dS = tau * S.diagonal()
    a_ij = np.asarray(A[rows, cols]).ravel()
    m_ij = np.asarray(Meps[rows, cols]).ravel()
    s_ij = tau * np.asarray(S[rows, cols]).ravel()
    rl = np.diff(A.indptr).astype(np.float64)
    absA = abs(A)
    off = np.asarray(absA.sum(axis=1)).ravel() / dA - 1.0
    ell = np.linalg.norm(edge_vec, axis=1)
    ti, tj = edge_vec[rows] / ell[rows, None], edge_vec[cols] / ell[cols, None]
    cosang = np.einsum("pd,pd->p", ti, tj)
    f = np.zeros((rows.size, F_IN))
    f[:, 0] = (rows == cols)
    f[:, 1] = a_ij / np.sqrt(dA[rows] * dA[cols])
    f[:, 2] = m_ij / np.sqrt(dM[rows] * dM[cols])
    f[:, 3] = s_ij / np.sqrt(dA[rows] * dA[cols])
    f[:, 4] = dS[rows] / dA[rows]
    f[:, 5] = dS[cols] / dA[cols]
    f[:, 6] = cosang
    f[:, 7] = np.log(ell[cols] / ell[rows])
    f[:, 8] = rl[rows] / 20.0
    f[:, 9] = rl[cols] / 20.0
    f[:, 10] = off[rows]
    f[:, 11] = off[cols]
    f[:, 12] = np.abs(f[:, 1])
    f[:, 13] = f[:, 1] ** 2
    f[:, 14] = f[:, 4] * f[:, 5]
    f[:, 15] = 1.0
    return f


def init_weights(seed=0):
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.normal(0, np.sqrt(2.0 / F_IN), (HID, F_IN)), "b1": np.zeros(HID),
        "W2": rng.normal(0, np.sqrt(2.0 / HID), (HID, HID)), "b2": np.zeros(HID),
        "W3": np.zeros((1, HID)), "b3": np.zeros(1),
    }


def mlp_forward(w, f):
    """Returns the output o (P,) and the activations needed by the backward pass."""
    z1 = f @ w["W1"].T + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(z2, 0.0)
    o = (h2 @ w["W3"].T + w["b3"]).ravel()
    return o, (f, z1, h1, z2, h2)


def mlp_backward(w, cache, d_o):
    """Gradients of sum(d_o * o) with respect to the weights."""
    f, z1, h1, z2, h2 = cache
    d_o = d_o[:, None]
    g = {"W3": d_o.T @ h2, "b3": d_o.sum(0)}
    dh2 = d_o @ w["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ w["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ f
    g["b1"] = dz1.sum(0)
    return g


S0 = float(np.log(np.e - 1.0))   # softplus(S0) = 1


def softplus(x):
    return np.logaddexp(0.0, x)


def factor(o, rows, cols, dA, n):
    """G (csr) and its values in entry order from the network output."""
    diag = rows == cols
    vals = np.where(diag, softplus(o + S0) / np.sqrt(dA[rows]), o / np.sqrt(dA[cols]))
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n)), vals


def kaporin_loss_grad_G(A, rows, cols, vals, V):
    """L and dL/dG (entry order) for probes V (n, P)."""
    n = A.shape[0]
    G = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    W = G.T @ V
    AW = A @ W
    nv = np.einsum("ik,ik->k", V, V)
    T = np.mean(np.einsum("ik,ik->k", W, AW) / nv)
    diag = rows == cols
    L = np.log(T) - 2.0 / n * np.sum(np.log(vals[diag]))
    dG = 2.0 / (V.shape[1] * T) * np.einsum("pk,pk->p", AW[cols] / nv, V[rows])
    dG[diag] -= 2.0 / n / vals[diag]
    return L, dG


def kaporin_loss_grad(w, A, feats, rows, cols, V):
    """L and its gradients with respect to the network weights."""
    n = A.shape[0]
    dA = A.diagonal()
    o, cache = mlp_forward(w, feats)
    _, vals = factor(o, rows, cols, dA, n)
    L, dG = kaporin_loss_grad_G(A, rows, cols, vals, V)
    diag = rows == cols
    sig = 1.0 / (1.0 + np.exp(-(o + S0)))
    d_o = np.where(diag, dG * sig / np.sqrt(dA[rows]), dG / np.sqrt(dA[cols]))
    return L, mlp_backward(w, cache, d_o), vals


def pair_energy_loss_grad(w, A, feats, rows, cols, B, X):
    """Energy-norm loss of the preconditioner on solver pairs (columns of B, X with A x = b):
        L_E = mean_k ||x_k - M b_k||_A^2 / ||x_k||_A^2,   M = G^T G,
    and its gradients with respect to the network weights. With v = x - G^T G b,
        dL_E/dG_ij = -(2/P) sum_k [(G b_k)_i (A v_k)_j + (G A v_k)_i (b_k)_j] / ||x_k||_A^2."""
    n = A.shape[0]
    dA = A.diagonal()
    o, cache = mlp_forward(w, feats)
    G, vals = factor(o, rows, cols, dA, n)
    GB = G @ B
    V = X - G.T @ GB
    AV = A @ V
    xAx = np.einsum("ik,ik->k", X, A @ X)
    P = B.shape[1]
    L = float(np.mean(np.einsum("ik,ik->k", V, AV) / xAx))
    GAV = G @ AV
    dG = -2.0 / P * (np.einsum("pk,pk,k->p", GB[rows], AV[cols], 1.0 / xAx)
                     + np.einsum("pk,pk,k->p", GAV[rows], B[cols], 1.0 / xAx))
    diag = rows == cols
    sig = 1.0 / (1.0 + np.exp(-(o + S0)))
    d_o = np.where(diag, dG * sig / np.sqrt(dA[rows]), dG / np.sqrt(dA[cols]))
    return L, mlp_backward(w, cache, d_o)


def energy_error(A, G, b, x):
    """||x - G^T G b||_A / ||x||_A per pair (columns of b, x)."""
    v = x - G.T @ (G @ b)
    return np.sqrt(np.einsum("ik,ik->k", v, A @ v) / np.einsum("ik,ik->k", x, A @ x))


def adam_step(w, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in w:
        m = state.setdefault("m_" + k, np.zeros_like(w[k]))
        v = state.setdefault("v_" + k, np.zeros_like(w[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        w[k] = w[k] - lr * mh / (np.sqrt(vh) + eps)


def pcg(A, b, apply_m, tol=1e-8, maxit=5000, x0=None):
    """Preconditioned CG with z = apply_m(r); stops at ||b - Ax|| <= tol ||b||."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    nb = np.linalg.norm(b)
    z = apply_m(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > tol * nb and it < maxit:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = apply_m(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it


STALL_WINDOW = 10        # iterations over which ||r|| must drop
STALL_DROP = 0.1         # by at least this fraction


def pcg_learned(A, b, apply_m, tol=1e-8, maxit=5000, x0=None):
    """Learned-preconditioner solve with the stall rule of the fallback: PCG with z = apply_m(r)
    stops as stalled when r.z <= 0 (M not positive definite on r), on non-finite values, or when
    ||r|| has not dropped by STALL_DROP over the last STALL_WINDOW iterations; Jacobi-PCG then
    restarts from the present iterate (from x0 after non-finite values). Returns x, the learned
    iterations, the Jacobi iterations and why the learned phase ended ("converged", "stalled",
    "nonfinite" or "cap")."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    start = x.copy()
    r = b - A @ x
    nb = np.linalg.norm(b)
    z = apply_m(r)
    rz = r @ z
    hist = [r @ r]
    why = "cap"
    it = 0
    p = z.copy()

    def state(rr, rz_, k):
        if not (np.isfinite(rr) and np.isfinite(rz_)):
            return "nonfinite"
        if rr <= (tol * nb) ** 2:
            return "converged"
        if not rz_ > 0 or (k >= STALL_WINDOW and rr > (1.0 - STALL_DROP) ** 2 * hist[k - STALL_WINDOW]):
            return "stalled"
        return None

    why = state(hist[0], rz, 0) or "cap"
    while why == "cap" and it < maxit:
        q = A @ p
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        z = apply_m(r)
        rz_new = r @ z
        it += 1
        hist.append(r @ r)
        s_ = state(hist[-1], rz_new, it)
        if s_:
            why = s_
            break
        p = z + (rz_new / rz) * p
        rz = rz_new
    if why == "converged":
        return x, it, 0, why
    dinv = 1.0 / A.diagonal()
    xj, it_j = pcg(A, b, lambda v: dinv * v, tol=tol, maxit=maxit, x0=start if why == "nonfinite" else x)
    return xj, it, it_j, why
