"""Learned preconditioner on the GPU vs the FP64 oracle (needs an MI355X).

Bars: G entries from the BF16-MFMA network within BF16 tolerance of the FP64 oracle on the same
weights; the Kaporin loss and its gradient from the GPU forward/backward kernels against the
oracle's (cosine >= 0.999, per-tensor relative <= 2e-2); GPU training cuts PCG iterations to
1e-8 versus Jacobi on held-out right-hand sides with the residual recomputed in FP64; a
non-finite network falls back to Jacobi and still converges.
"""
import numpy as np
import pytest

import qh_inputs as qi

from .gpu_setup import gpu_context
from .test_oracle_learned import edge_problem

pytestmark = pytest.mark.gpu

N = 5
DT = 10 * 7.69e-10 / N


@pytest.fixture(scope="module")
def prob():
    A, rows, cols, f = edge_problem(N)
    mesh = qi.BoxMesh(N)
    return mesh, A, rows, cols, f


def _weights(seed):
    from oracle import learned as Lr
    w = Lr.init_weights(seed)
    rng = np.random.default_rng(seed + 10)
    w["W3"] = rng.normal(0, 0.1, w["W3"].shape)
    w["b1"] = rng.normal(0, 0.1, w["b1"].shape)
    w["b2"] = rng.normal(0, 0.1, w["b2"].shape)
    w["b3"] = rng.normal(0, 0.05, w["b3"].shape)
    return w


def _flat(w):
    return np.concatenate([w["W1"].ravel(), w["b1"], w["W2"].ravel(), w["b2"], w["W3"].ravel(), w["b3"]]).astype(np.float32)


def _unflat(v):
    return {"W1": v[:1024].reshape(64, 16), "b1": v[1024:1088], "W2": v[1088:5184].reshape(64, 64),
            "b2": v[5184:5248], "W3": v[5248:5312].reshape(1, 64), "b3": v[5312:5313]}


def test_factor_matches_oracle(prob):
    from oracle import learned as Lr
    mesh, A, rows, cols, f = prob
    ctx = gpu_context(mesh, DT)
    w = _weights(1)
    # the oracle runs on the float32-rounded weights the GPU receives
    w32 = _unflat(_flat(w).astype(np.float64))
    ctx.precond_set_weights(_flat(w))
    gr, gc, gv = ctx.precond_factor()
    assert np.array_equal(gr, rows) and np.array_equal(gc, cols)
    o, _ = Lr.mlp_forward(w32, f)
    _, ref = Lr.factor(o, rows, cols, A.diagonal(), A.shape[0])
    scale = np.where(rows == cols, 1.0 / np.sqrt(A.diagonal()[rows]), 1.0 / np.sqrt(A.diagonal()[cols]))
    err = np.abs(gv - ref) / scale                    # error in units of the network output
    assert err.max() < 0.05 * max(1.0, np.abs(o).max())
    assert np.corrcoef(gv, ref)[0, 1] > 0.9999


def _bf16(x):
    """Round to the nearest BF16 value (ties to even), the operand precision of the MFMA layers."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_loss_and_gradient_match_oracle(prob):
    from oracle import learned as Lr
    mesh, A, rows, cols, f = prob
    ctx = gpu_context(mesh, DT)
    w = _weights(2)
    w32 = _unflat(_flat(w).astype(np.float64))
    ctx.precond_set_weights(_flat(w))
    V = np.sign(np.random.default_rng(3).standard_normal((A.shape[0], 16))).astype(np.float32)
    loss_g, grad_g = ctx.precond_loss_grad(V)
    gg = grad_g.astype(np.float64)
    # against the FP64 oracle on exact features: direction of the gradient and the loss
    loss_o, grad_o, _ = Lr.kaporin_loss_grad(w32, A, f, rows, cols, V.astype(np.float64))
    assert abs(loss_g - loss_o) < 2e-2 * max(1.0, abs(loss_o))
    go = _flat(grad_o).astype(np.float64)
    assert gg @ go / (np.linalg.norm(gg) * np.linalg.norm(go)) >= 0.999
    # against the FP64 oracle on the BF16 inputs the kernels consume (features, weight
    # matrices): per tensor within 2e-2
    wb = dict(w32, W1=_bf16(w32["W1"]), W2=_bf16(w32["W2"]))
    loss_b, grad_b, _ = Lr.kaporin_loss_grad(wb, A, _bf16(f), rows, cols, V.astype(np.float64))
    gb = _flat(grad_b).astype(np.float64)
    assert gg @ gb / (np.linalg.norm(gg) * np.linalg.norm(gb)) >= 0.999
    for k in ("W1", "W2", "W3", "b1", "b2"):
        a, b = _unflat(gg)[k].ravel(), np.asarray(grad_b[k]).ravel()
        assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b) + 1e-12, k


def _edge_rhs(A, k, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((A.shape[0], k))
    return (A @ X).T.copy(), X.T.copy()


def test_training_beats_jacobi_iterations(prob):
    import paper_2103_06737_amd as qh
    mesh, A, rows, cols, f = prob
    ctx = gpu_context(mesh, DT)
    rhs, sol = _edge_rhs(A, 2, 5)
    st = ctx.precond_train(steps=150, lr=3e-3, seed=1, validate_every=25, rhs=rhs, sol=sol)
    assert st["loss_last"] < st["loss_first"]
    assert st["val_iters_best"] < st["val_iters_jacobi"]
    bt, xt = _edge_rhs(A, 3, 99)
    for k in range(3):
        xl, sl = ctx.field_solve(qh.SYS_EDGE, bt[k], tol=1e-8, precond=qh.PC_LEARNED)
        xj, sj = ctx.field_solve(qh.SYS_EDGE, bt[k], tol=1e-8, precond=qh.PC_JACOBI)
        assert sl["res"] <= 1e-8 and sl["fallback"] == 0
        assert np.linalg.norm(A @ xl - bt[k]) <= 1.0001e-8 * np.linalg.norm(bt[k])
        assert sl["iters"] <= 0.75 * sj["iters"], (sl, sj)


def test_nonfinite_network_falls_back_to_jacobi(prob):
    import paper_2103_06737_amd as qh
    mesh, A, rows, cols, f = prob
    ctx = gpu_context(mesh, DT)
    w = _flat(_weights(4))
    w[5312] = np.nan
    ctx.precond_set_weights(w)
    b, _ = _edge_rhs(A, 1, 7)
    x, st = ctx.field_solve(qh.SYS_EDGE, b[0], tol=1e-8, precond=qh.PC_LEARNED, max_it=400)
    assert st["fallback"] == 1 and st["res"] <= 1e-8
    assert np.linalg.norm(A @ x - b[0]) <= 1.0001e-8 * np.linalg.norm(b[0])


def test_full_cycle_with_learned_preconditioner(prob):
    import paper_2103_06737_amd as qh
    from oracle.complex_ import Complex
    mesh, A, rows, cols, f = prob
    ctx = gpu_context(mesh, DT)
    ctx.precond_train(steps=80, lr=3e-3, seed=2, validate_every=0)
    mi = ctx.mesh_info()
    ctx.fields_init_synthetic(qi.white(mi.n_edges, 0, 3), qi.white(mi.n_edges, 0, 5), 1e3, 0.1, 1e-3)
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    parts = qi.uniform_plasma(mesh, 5000, 1e6, seed=0)
    ctx.particles_upload(sid, *parts)
    cx = Complex(mesh.xyz, mesh.tets)
    for pc in (qh.PC_LEARNED, qh.PC_JACOBI):
        p = ctx.step_params(field_mode=qh.FIELDS_SOLVE, precond=pc, verify=1)
        for st in ctx.pic_step(p, 3):
            assert st["continuity_bad"] == 0 and st["divb_bad"] == 0
            assert st["edge_res"] <= 1e-8 and st["gauss_res"] <= 1e-8 and st["fallbacks"] == 0
    e, b = ctx.fields_download()
    assert not (cx.D @ b).any()


def test_save_and_load_keep_the_preconditioner(prob):
    """A trained network saved as a blob and loaded into a fresh context (the same mesh, and a
    jittered one: the network does not depend on the mesh) gives the same factor bit for bit and
    the same solve; a blob with a flipped byte, a short one and one of another size are refused
    and leave the loaded network in place."""
    import paper_2103_06737_amd as qh
    mesh, A, rows, cols, f = prob
    ctx = gpu_context(mesh, DT)
    ctx.precond_train(steps=40, lr=3e-3, seed=3, validate_every=0)
    blob = ctx.precond_save()
    assert blob[:8] == b"QHPRECND" and len(blob) == 16 + 4 * qh.MLP_NPARAM + 4
    _, _, v0 = ctx.precond_factor()
    rhs = np.random.default_rng(4).standard_normal(A.shape[0])
    _, s0 = ctx.field_solve(qh.SYS_EDGE, rhs, tol=1e-8, precond=qh.PC_LEARNED)
    ctx2 = gpu_context(mesh, DT)
    ctx2.precond_load(blob)
    _, _, v1 = ctx2.precond_factor()
    assert np.array_equal(v0, v1)
    _, s1 = ctx2.field_solve(qh.SYS_EDGE, rhs, tol=1e-8, precond=qh.PC_LEARNED)
    assert s1["iters"] == s0["iters"]
    bad = bytearray(blob)
    bad[100] ^= 1
    for wrong in (bytes(bad), blob[:-10], blob[:12]):
        with pytest.raises(qh.QhError) as ei:
            ctx2.precond_load(wrong)
        assert ei.value.code == qh.QH_EINVAL
    _, _, v2 = ctx2.precond_factor()
    assert np.array_equal(v0, v2)
    jm = qi.make_mesh(qi.CONFIGS["jitter4"])
    ctx3 = gpu_context(jm, 1e-11)
    ctx3.precond_load(blob)
    assert np.array_equal(ctx3.precond_get_weights(), ctx.precond_get_weights())
