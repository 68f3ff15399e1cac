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

from .gpu_setup import gpu_context, record as _record
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


def _bf16(x):
    """Round to the nearest BF16 value (ties to even), the operand precision of the MFMA layers."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


U32 = 2.0 ** -24          # FP32 unit roundoff
ULP_BF16 = 2.0 ** -7      # spacing of BF16 values relative to their magnitude (at most)


def factor_model(w32, f, rows, cols, dA):
    """Error model of the factor kernel. The network as the kernel evaluates it: features, W1 and
    W2 rounded to BF16 (the MFMA operands), the first layer's activations rounded to BF16 before
    the second layer, biases, W3 and every sum exact here; G = o / sqrt(A_jj) off the diagonal,
    softplus(o + s0) / sqrt(A_ii) on it. Returns G of this model and a per-entry bound on what
    the kernel may add to it: FP32 sums of k terms err by at most k u |terms| (u = 2^-24, any
    order; the BF16 products are exact in FP32), an error e in a first-layer activation can move
    its BF16 rounding by e plus one BF16 spacing (2^-7 of its size), ReLU is 1-Lipschitz, and the
    FP32 scale, multiply and softplus add a few units of 2^-24 of G."""
    from oracle import learned as Lr
    xb, W1b, W2b = _bf16(f), _bf16(w32["W1"]), _bf16(w32["W2"])
    b1, b2, w3, b3 = w32["b1"], w32["b2"], w32["W3"].ravel(), w32["b3"][0]
    z1 = xb @ W1b.T + b1
    h1 = _bf16(np.maximum(z1, 0.0))
    z2 = h1 @ W2b.T + b2
    h2 = np.maximum(z2, 0.0)
    o = h2 @ w3 + b3
    e1 = 17 * U32 * (np.abs(xb) @ np.abs(W1b).T + np.abs(b1))
    d1 = e1 + ULP_BF16 * (np.abs(h1) + e1)
    e2 = 65 * U32 * (np.abs(h1) @ np.abs(W2b).T + np.abs(b2)) + d1 @ np.abs(W2b).T
    eo = 65 * U32 * (np.abs(h2) @ np.abs(w3) + abs(b3)) + e2 @ np.abs(w3)
    diag = rows == cols
    scale = np.where(diag, 1.0 / np.sqrt(dA[rows]), 1.0 / np.sqrt(dA[cols]))
    G = np.where(diag, Lr.softplus(o + Lr.S0), o) * scale
    # softplus' <= 1; the FP32 scale differs from 1/sqrt by half a unit; FP32 log1p(exp) a few units
    bound = eo * scale + 16 * U32 * np.abs(G) + 1e-30
    return G, bound


def test_factor_matches_oracle(prob):
    """G from the BF16-MFMA network against the FP64 oracle on the same FP32 weights, with a
    tolerance derived from the kernel's precision: every entry within the bound of factor_model
    around the model of the kernel's roundings; the effect of the BF16 rounding itself (model
    against the exact oracle) is recorded."""
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
    Gm, bound = factor_model(w32, f, rows, cols, A.diagonal())
    dev = np.abs(gv - Gm)
    assert (dev <= bound).all(), (dev / bound).max()
    # nearly every entry sits within the FP32 rounding of the sums: the BF16 roundings of the
    # activations rarely move
    assert np.quantile(dev / np.abs(Gm).max(), 0.99) < 1e-5
    assert np.corrcoef(gv, ref)[0, 1] > 0.9999
    _record("factor_5cube", dict(
        kernel_vs_model_max_rel=float(dev.max() / np.abs(Gm).max()),
        kernel_vs_model_max_over_bound=float((dev / bound).max()),
        model_vs_exact_max_rel=float(np.abs(Gm - ref).max() / np.abs(ref).max()),
        kernel_vs_exact_max_rel=float(np.abs(gv - ref).max() / np.abs(ref).max()),
        kernel_vs_exact_p99_rel=float(np.quantile(np.abs(gv - ref) / np.abs(ref).max(), 0.99))))


def test_preconditioner_application_matches_oracle(prob):
    """z = G^T (G r) from the application kernels (through qh_precond_apply) element by element:
    (1) against the oracle's FP64 factor of the same weights, within the bound that the factor's
    error model and the BF16 copies the application reads (half a BF16 spacing, 2^-8, of each
    entry) give through |G|^T |dG| |r| + |dG|^T |G| |r| + |dG|^T |dG| |r|; (2) against the same
    products done in FP64 on the host from the factor the kernels hold, rounded to BF16, within
    the FP64 rounding of the sums (the application's own arithmetic)."""
    import scipy.sparse as sp
    from oracle import learned as Lr
    mesh, A, rows, cols, f = prob
    n = A.shape[0]
    ctx = gpu_context(mesh, DT)
    w = _weights(5)
    w32 = _unflat(_flat(w).astype(np.float64))
    ctx.precond_set_weights(_flat(w))
    rng = np.random.default_rng(11)
    o, _ = Lr.mlp_forward(w32, f)
    G, gref = Lr.factor(o, rows, cols, A.diagonal(), n)
    Gm, bound = factor_model(w32, f, rows, cols, A.diagonal())
    dG = sp.csr_matrix((np.abs(Gm - gref) + bound + 2.0 ** -8 * (np.abs(Gm) + bound), (rows, cols)), shape=(n, n))
    aG = abs(G)
    for k in range(3):
        r = rng.standard_normal(n) * (1.0 if k < 2 else 1e-12)
        z = ctx.precond_apply(r)
        zo = G.T @ (G @ r)
        ar = np.abs(r)
        tol = aG.T @ (dG @ ar) + dG.T @ (aG @ ar) + dG.T @ (dG @ ar) + 1e-13 * (aG.T @ (aG @ ar))
        assert (np.abs(z - zo) <= tol).all()
        _, _, gv = ctx.precond_factor()
        Gb = sp.csr_matrix((_bf16(gv), (rows, cols)), shape=(n, n))
        zb = Gb.T @ (Gb @ r)
        aGb = abs(Gb)
        assert (np.abs(z - zb) <= 64 * np.finfo(float).eps * (aGb.T @ (aGb @ ar))).all()
        if k == 0:
            _record("prec_apply_5cube", dict(
                vs_oracle_max_rel=float(np.abs(z - zo).max() / np.abs(zo).max()),
                vs_oracle_max_over_bound=float((np.abs(z - zo) / tol).max()),
                vs_own_factor_max_rel=float(np.abs(z - zb).max() / np.abs(zb).max())))
    # a zero network is Jacobi: z = bf16(fl32(1 / sqrt(A_ii)))^2 r within the FP32 softplus(s0) = 1
    ctx.precond_set_weights(_flat(Lr.init_weights(0)))
    r = rng.standard_normal(n)
    z = ctx.precond_apply(r)
    assert np.allclose(z, r / A.diagonal(), rtol=2 ** -6, atol=0)


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
    rec = {}
    for k in ("W1", "W2", "W3", "b1", "b2"):
        a, b = _unflat(gg)[k].ravel(), np.asarray(grad_b[k]).ravel()
        ex = np.asarray(grad_o[k]).ravel()
        # the kernels' own arithmetic (BF16 activations and gradient operands, FP32 sums): within
        # 2e-2 per tensor of the oracle fed the kernels' BF16 inputs
        assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b) + 1e-12, k
        # against the oracle on exact inputs the error of rounding the inputs to BF16 adds to it;
        # the oracle measures that part itself (triangle inequality)
        inp = np.linalg.norm(b - ex)
        assert np.linalg.norm(a - ex) <= inp + 2e-2 * np.linalg.norm(ex) + 1e-12, k
        rec[k] = dict(kernel_vs_bf16_inputs=float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                      bf16_inputs_vs_exact=float(inp / np.linalg.norm(ex)),
                      kernel_vs_exact=float(np.linalg.norm(a - ex) / np.linalg.norm(ex)))
    _record("gradient_5cube", rec)


def test_pair_loss_and_gradient_match_oracle(prob):
    """The energy-norm loss on 16 solver pairs (A x = b, x random) and its weight gradient from the
    GPU kernels (pairs stored in FP32, network in BF16) against the FP64 oracle: loss within 2e-2,
    gradient direction (cosine >= 0.999), per tensor within 2e-2 of the oracle fed the kernels' BF16
    inputs and FP32 pairs, and against the exact oracle within that plus the inputs' rounding
    effect, measured by the oracle."""
    from oracle import learned as Lr
    mesh, A, rows, cols, f = prob
    ctx = gpu_context(mesh, DT)
    w = _weights(7)
    w32 = _unflat(_flat(w).astype(np.float64))
    ctx.precond_set_weights(_flat(w))
    X = np.random.default_rng(17).standard_normal((A.shape[0], 16))
    B = A @ X
    ctx.pairs_record(16)
    ctx.pairs_add(B.T.copy(), X.T.copy())
    assert ctx.pairs_count() == 16
    loss_g, grad_g = ctx.precond_pair_loss_grad(np.arange(16))
    gg = grad_g.astype(np.float64)
    loss_o, grad_o = Lr.pair_energy_loss_grad(w32, A, f, rows, cols, B, X)
    assert abs(loss_g - loss_o) <= 2e-2 * loss_o
    go = _flat(grad_o).astype(np.float64)
    assert gg @ go / (np.linalg.norm(gg) * np.linalg.norm(go)) >= 0.999
    B32, X32 = B.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64)
    wb = dict(w32, W1=_bf16(w32["W1"]), W2=_bf16(w32["W2"]))
    _, grad_b = Lr.pair_energy_loss_grad(wb, A, _bf16(f), rows, cols, B32, X32)
    rec = {"loss_rel": abs(loss_g - loss_o) / loss_o}
    for k in ("W1", "W2", "W3", "b1", "b2"):
        a, b = _unflat(gg)[k].ravel(), np.asarray(grad_b[k]).ravel()
        ex = np.asarray(grad_o[k]).ravel()
        assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b) + 1e-12, k
        inp = np.linalg.norm(b - ex)
        assert np.linalg.norm(a - ex) <= inp + 2e-2 * np.linalg.norm(ex) + 1e-12, k
        rec[k] = dict(kernel_vs_bf16_inputs=float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                      bf16_inputs_vs_exact=float(inp / np.linalg.norm(ex)))
    _record("pair_gradient_5cube", rec)


def test_training_on_recorded_solver_pairs(prob):
    """Pairs the plain solver generates during a full cycle (5^3 box, 5000 electrons, Jacobi,
    recorded by the step into the device bank) in the training objective with weight 0.5, held-out
    pairs of another particle seed validating: fewer PCG iterations than Jacobi, the pairs'
    energy-norm loss falls, and the kept network's energy-norm error on the held-out pairs is
    reported."""
    import paper_2103_06737_amd as qh
    mesh, A, rows, cols, f = prob

    def cycle_ctx(seed):
        # no random part in B: its curl would drive 1e6 V/m waves that push electrons past c
        # within a few steps (then past the walk cap), as the oracle's cycle shows too
        c = gpu_context(mesh, DT)
        mi = c.mesh_info()
        c.fields_init_synthetic(qi.white(mi.n_edges, seed, 3), qi.white(mi.n_edges, seed, 5), 1e3, 0.1, 0.0)
        sid = c.species_add(-qi.QE / qi.ME, -1)
        c.particles_upload(sid, *qi.uniform_plasma(mesh, 5000, 1e6, seed=seed))
        return c

    prm = qh.Context.step_params(field_mode=qh.FIELDS_SOLVE, precond=qh.PC_JACOBI)
    val = cycle_ctx(0)
    rhs, sol = [], []
    for _ in range(2):
        val.pic_step(prm)
        r, x = val.edge_system_download()
        rhs.append(r)
        sol.append(x)
    ctx = cycle_ctx(1)
    ctx.pairs_record(40)
    ctx.pic_step(prm, 45)
    assert ctx.pairs_count() == 40
    st = ctx.precond_train(steps=150, lr=3e-3, seed=3, validate_every=25, rhs=np.array(rhs), sol=np.array(sol),
                           pair_weight=0.5)
    assert st["val_iters_best"] < 0.75 * st["val_iters_jacobi"], st
    assert 0 < st["pair_loss_last"] < st["pair_loss_first"], st
    assert 0 < st["val_energy_err"] < 1.0, st
    _record("train_pairs_5cube", st)


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
    for solver in (qh.SOLVER_FP64, qh.SOLVER_MIXED):
        x, st = ctx.field_solve(qh.SYS_EDGE, b[0], tol=1e-8, precond=qh.PC_LEARNED, max_it=400, solver=solver)
        assert st["fallback"] == 1 and st["res"] <= 1e-8
        assert np.linalg.norm(A @ x - b[0]) <= 1.0001e-8 * np.linalg.norm(b[0])


def test_stalled_network_falls_back_quickly(prob):
    """Finite but bad weights (outputs up to ~170: G badly conditioned, M = G^T G still SPD): the
    stall rule (||r|| not 10 % lower over 10 iterations) ends the learned phase long before the
    iteration cap, and Jacobi-PCG restarted from its iterate reaches 1e-8; a trained network in
    the same call sequence does not trip it."""
    import paper_2103_06737_amd as qh
    from .test_oracle_learned import _bad_weights
    mesh, A, rows, cols, f = prob
    ctx = gpu_context(mesh, DT)
    ctx.precond_set_weights(_flat(_bad_weights()))
    b, _ = _edge_rhs(A, 1, 7)
    _, sj = ctx.field_solve(qh.SYS_EDGE, b[0], tol=1e-8, precond=qh.PC_JACOBI, max_it=2000)
    for solver in (qh.SOLVER_FP64, qh.SOLVER_MIXED):
        x, st = ctx.field_solve(qh.SYS_EDGE, b[0], tol=1e-8, precond=qh.PC_LEARNED, max_it=2000, solver=solver)
        assert st["fallback"] == 1 and st["res"] <= 1e-8
        assert st["iters"] < sj["iters"] + 200        # without the rule: 2000 learned iterations first
        assert np.linalg.norm(A @ x - b[0]) <= 1.0001e-8 * np.linalg.norm(b[0])
    from oracle import learned as Lr
    ctx.precond_set_weights(_flat(Lr.init_weights(0)))
    ctx.precond_train(steps=80, lr=3e-3, seed=2, validate_every=0)
    _, sl = ctx.field_solve(qh.SYS_EDGE, b[0], tol=1e-8, precond=qh.PC_LEARNED, max_it=2000)
    assert sl["fallback"] == 0 and sl["res"] <= 1e-8


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
        for solver in (qh.SOLVER_FP64, qh.SOLVER_MIXED):
            p = ctx.step_params(field_mode=qh.FIELDS_SOLVE, precond=pc, verify=1, solver=solver)
            for st in ctx.pic_step(p, 3):
                assert st["continuity_bad"] == 0 and st["divb_bad"] == 0
                assert st["edge_res"] <= 1e-8 and st["gauss_res"] <= 1e-8 and st["fallbacks"] == 0
                assert (st["edge_refinements"] >= 1) == (solver == qh.SOLVER_MIXED)
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
