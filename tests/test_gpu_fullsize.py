"""The HIP path at full workload size, in the launch configuration the benchmark times (needs an
MI355X). The oracle checks what it can afford at this size: every integer deposit (re-deposited
from the GPU's own pieces, bit for bit), continuity and D b on the host, sampled particles pushed
one by one, and the field update step by step: the edge right-hand side, the solution's residual
with its own FP64 matrix, the Gauss-law residual and the integer Faraday update.

Workloads (sizes as quoted): 64^3 Kuhn cube with 16M electrons, full implicit cycle with the
learned preconditioner; 32^3 Kuhn cube with a 1M-electron beam in frozen random fields for 200
steps; the 96^3 graded mesh with two species (particle count reduced to 2M + 2M).
"""
import numpy as np
import pytest

import qh_inputs as qi

from .gpu_setup import (GATHER_REL, PUSH_V_REL, PUSH_X_ABS, S, err_stats, gpu_context, oracle_fields,
                        oracle_setup, record)

pytestmark = pytest.mark.gpu

U_B = 2.0 ** -56


@pytest.fixture(scope="module")
def plasma64():
    cfg = qi.CONFIGS["plasma64"]
    mesh = qi.make_mesh(cfg)
    parts = qi.make_particles(mesh, cfg)
    cx, op, po = oracle_setup(mesh)
    return cfg, mesh, parts, cx, op, po


@pytest.mark.parametrize("solver", ["mixed", "fp64"])
def test_plasma64_full_cycle(plasma64, solver):
    """One step of the 64^3 / 16M cycle in the launch configuration the benchmark times (learned
    preconditioner; the mixed-precision edge solve of its headline run, and the FP64 one), checked
    piece by piece against the oracle."""
    import paper_2103_06737_amd as qh
    from oracle.field import FieldOracle
    cfg, mesh, parts, cx, op, po = plasma64
    dt, weight = cfg["dt"], cfg["weight"]
    u_q = qi.QE * weight * 2.0 ** -40
    ctx = gpu_context(mesh, dt, weight=weight)
    ctx.fields_init_synthetic(qi.white(cx.Ne, 0, 3), qi.white(cx.Ne, 0, 5), cfg["sigma_e"], cfg["bz"],
                              cfg["sigma_b"])
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    x, v, tet = parts["e"]
    n = tet.size
    assert n == 16_000_000
    ctx.particles_upload(sid, x, v, tet)
    ctx.charge_background(1)
    ctx.precond_train(steps=60, lr=3e-3, seed=1, validate_every=0)
    # every product tile of A, G and G^T on this mesh fits four 2^14-column windows: all 16-bit
    mi = ctx.mesh_info()
    assert mi.nnz_edge_c16 == mi.nnz_edge and mi.nnz_factor_c16 == 2 * mi.nnz_factor > 0
    e0, b0 = ctx.fields_download()
    _, Q0 = ctx.deposits_download()
    ctx.capture_segments(int(1.5 * n))
    params = ctx.step_params(field_mode=qh.FIELDS_SOLVE, precond=qh.PC_LEARNED, sort_every=20, verify=1,
                             solver=qh.SOLVER_MIXED if solver == "mixed" else qh.SOLVER_FP64)
    st = ctx.pic_step(params)[0]
    assert (st["edge_refinements"] >= 1) == (solver == "mixed")
    assert st["continuity_bad"] == 0 and st["divb_bad"] == 0 and st["lost"] == 0
    assert st["fallbacks"] == 0 and st["edge_res"] <= 1e-8 and st["gauss_res"] <= 1e-8
    assert st["crossings"] > 100_000
    g, Q1 = ctx.deposits_download()
    e1, b1 = ctx.fields_download()
    xg, vg, tg = ctx.particles_download(sid)

    # continuity on the host, bit for bit
    assert np.array_equal(cx.G.T @ g, Q1 - Q0)
    # the GPU's own pieces, re-deposited by the oracle, give its g and Q bit for bit
    nseg, seg = ctx.segments_download()
    assert nseg == seg["tet"].size and nseg >= n
    g_re, _ = po.deposit_list(seg["tet"], seg["lam0"], seg["lam1"], -np.ones(nseg), np.zeros(0),
                              np.zeros((0, 4)), np.zeros(0))
    assert np.array_equal(g_re, g)
    order = np.lexsort((seg["seq"], seg["pid"]))
    pid = seg["pid"][order]
    last = np.r_[pid[1:] != pid[:-1], True]
    assert last.sum() == n
    _, Q_re = po.deposit_list(np.zeros(0), np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0),
                              seg["tet"][order][last], seg["lam1"][order][last], -np.ones(n))
    assert np.array_equal(Q_re, Q1)
    assert (seg["lam0"].sum(1) == S).all() and (seg["lam1"].sum(1) == S).all()

    # device point location of a million of the particles' start points: the generator's tet but
    # for points on a face up to the FP32 rounding of barycentrics (|grad lambda| up to 110/m
    # times a coordinate spacing of 6e-8 m near 1 m: 7e-6), which may get the neighbour
    tl = ctx.locate(x[:1_000_000].astype(np.float64))
    assert (tl >= 0).all()
    mism = np.flatnonzero(tl != tet[:1_000_000])
    assert mism.size < 1000
    lm = np.einsum("pij,pj->pi", op.Minv[tl[mism]], np.column_stack([np.ones(mism.size), x[mism].astype(np.float64)]))
    assert lm.min() > -1e-5

    # sampled particles pushed one by one by the oracle through the same start fields
    idx = np.random.default_rng(7).choice(n, 4096, replace=False)
    orc = po.push(e0, b0 * U_B, x[idx], v[idx], tet[idx], -qi.QE / qi.ME, dt, -1)
    same = tg[idx] == orc["tet"]
    assert same.mean() > 0.999
    assert np.abs(xg[idx] - orc["x"]).max(axis=1)[same].max() <= PUSH_X_ABS
    assert (np.abs(vg[idx] - orc["v"]).max(axis=1)[same] / np.abs(orc["v"]).max()).max() <= PUSH_V_REL
    # the FP32 gather (the push's per-tet records, read through the probe) against FP64 at the
    # sampled particles' new points in the new fields
    e1p, b1p = ctx.fields_download()
    Ep, Bp = ctx.probe_fields(xg[idx].astype(np.float64), tg[idx])
    Eo, Bo = po.gather(e1p, b1p * U_B, xg[idx].astype(np.float64), tg[idx])
    assert np.abs(Ep - Eo).max() <= GATHER_REL * np.abs(Eo).max()
    assert np.abs(Bp - Bo).max() <= GATHER_REL * np.abs(Bo).max()
    record("plasma64_one_step", dict(
        E_rel=err_stats(np.abs(Ep - Eo).max(axis=1) / np.abs(Eo).max()),
        B_rel=err_stats(np.abs(Bp - Bo).max(axis=1) / np.abs(Bo).max()),
        x_abs_m=err_stats(np.abs(xg[idx] - orc["x"]).max(axis=1)[same]),
        v_rel=err_stats(np.abs(vg[idx] - orc["v"]).max(axis=1)[same] / np.abs(orc["v"]).max()),
        same_tet=float(same.mean())))

    # the field update of this step, piece by piece against the oracle's FP64 operators:
    # right-hand side of the edge system (same sums, another order), the solution's residual,
    # the discrete Gauss law after the correction, and the integer Faraday update bit for bit
    fo = FieldOracle(cx, op, dt)
    rhs, sol = ctx.edge_system_download()
    b_real, g_real = b0.astype(np.float64) * U_B, g.astype(np.float64) * u_q
    rhs_o = fo.rhs(e0, b_real, g_real)
    # the terms cancel strongly (a uniform B has no discrete curl): bound the difference row by
    # row by the rounding of sums of |terms| (64 ulps of the absolute sum)
    terms = (abs(fo.Bm) @ np.abs(e0) + dt * (abs(op.CtMmu) @ np.abs(b_real)) + np.abs(g_real))[cx.int_edges]
    assert (np.abs(rhs - rhs_o) <= 64 * np.finfo(float).eps * terms).all()
    assert np.linalg.norm(fo.A @ sol - rhs_o) <= 1.001e-8 * np.linalg.norm(rhs_o)
    rho = u_q * (Q0 - Q1).astype(np.float64)[cx.int_nodes]   # Q_bg = Q0
    assert fo.gauss_error(e1, rho) <= 1.01e-8
    u = np.rint((0.5 * dt / U_B) * (e1 + e0)).astype(np.int64)
    assert np.array_equal(b1, b0 - cx.C @ u)
    assert np.array_equal(cx.D @ b1, cx.D @ b0)

    # quasi-Helmholtz split of the new field (Sec. III): rho_bar is the discrete divergence (the
    # charge, by the Gauss law just enforced), E_s + G E_ns = e and E_s has no divergence
    e_ns, e_s, rho_bar, st = ctx.fields_decompose(tol=1e-10)
    div = (fo.GtMeps @ e1)[cx.int_nodes]
    absd = (abs(fo.GtMeps) @ np.abs(e1))[cx.int_nodes]
    assert (np.abs(rho_bar[cx.int_nodes] - div) <= 64 * np.finfo(float).eps * absd).all()
    assert np.abs(cx.G.astype(float) @ e_ns + e_s - e1).max() <= 1e-12 * np.abs(e1).max()
    assert np.linalg.norm((fo.GtMeps @ e_s)[cx.int_nodes]) <= 1e-9 * np.linalg.norm(absd)
    assert np.linalg.norm(rho_bar[cx.int_nodes] - rho) <= 1.01e-8 * (np.linalg.norm(rho) + np.linalg.norm(absd))


def test_plasma64_100_steps(plasma64):
    """The workload's full run: 100 steps of the 64^3 / 16M cycle with the learned preconditioner
    (mixed-precision edge solve, as the benchmark runs it) and a re-sort every 20 steps, every invariant checked on the device at every step (continuity
    bit for bit, D b unchanged, no lost particle, no fallback, both residuals at 1e-8); at the end
    the total charge is the initial one, D b is unchanged on the host and sampled particles lie
    in the tets the device holds them in."""
    import paper_2103_06737_amd as qh
    cfg, mesh, parts, cx, op, po = plasma64
    ctx = gpu_context(mesh, cfg["dt"], weight=cfg["weight"])
    ctx.fields_init_synthetic(qi.white(cx.Ne, 0, 3), qi.white(cx.Ne, 0, 5), cfg["sigma_e"], cfg["bz"],
                              cfg["sigma_b"])
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    x, v, tet = parts["e"]
    ctx.particles_upload(sid, x, v, tet)
    ctx.charge_background(1)
    ctx.precond_train(steps=30, lr=3e-3, seed=1, validate_every=0)
    _, b0 = ctx.fields_download()
    _, Q0 = ctx.deposits_download()
    params = ctx.step_params(field_mode=qh.FIELDS_SOLVE, precond=qh.PC_LEARNED, sort_every=cfg["sort_every"],
                             verify=1, solver=qh.SOLVER_MIXED)
    stats = ctx.pic_step(params, cfg["steps"])
    assert len(stats) == 100
    for k, st in enumerate(stats):
        assert st["continuity_bad"] == 0 and st["divb_bad"] == 0 and st["lost"] == 0, (k, st)
        assert st["fallbacks"] == 0 and st["edge_res"] <= 1e-8 and st["gauss_res"] <= 1e-8, (k, st)
    assert sum(st["crossings"] for st in stats) > 100 * 100_000
    _, Q1 = ctx.deposits_download()
    _, b1 = ctx.fields_download()
    assert Q1.sum() == Q0.sum()
    assert np.array_equal(cx.D @ b1, cx.D @ b0)
    xg, _, tg = ctx.particles_download(sid)
    assert tg.size == tet.size and (tg >= 0).all()
    idx = np.random.default_rng(9).choice(tg.size, 200_000, replace=False)
    lam = np.einsum("pij,pj->pi", op.Minv[tg[idx]], np.column_stack([np.ones(idx.size), xg[idx].astype(np.float64)]))
    assert lam.min() > -1e-5
    ctx.close()


def test_plasma64_preconditioner_application_sampled_rows(plasma64):
    """The learned preconditioner's application z = G^T (G r) on the 64^3 edge system (1.8 M
    rows) in the launch configuration of the cycle, on 512 sampled rows: against the oracle's
    FP64 factor of the same weights, built only on the rows those outputs need (the rows k with
    G_ki != 0 for a sampled i, each whole), within the bound of the factor's error model; and
    against FP64 products of the kernels' own factor rounded to BF16, within the rounding of
    the sums."""
    import scipy.sparse as sp
    from oracle import learned as Lr
    from .test_gpu_learned import _bf16, _flat, _unflat, _weights, factor_model
    cfg, mesh, parts, cx, op, po = plasma64
    dt = cfg["dt"]
    tau = dt * dt / 4
    ctx = gpu_context(mesh, dt, weight=cfg["weight"])
    w = _weights(6)
    w32 = _unflat(_flat(w).astype(np.float64))
    ctx.precond_set_weights(_flat(w))
    ie = cx.int_edges
    Me = op.Meps[ie][:, ie].tocsr()
    Sm = op.S[ie][:, ie].tocsr()
    A = (Me + tau * Sm).tocsr()
    n = A.shape[0]
    rng = np.random.default_rng(12)
    r = rng.standard_normal(n)
    z = ctx.precond_apply(r)
    sample = np.sort(rng.choice(n, 512, replace=False))
    L = sp.tril(A, format="csr")
    LT = L.T.tocsr()                      # row i of L^T: the rows k >= i with L_ki != 0
    need = np.unique(np.concatenate([LT.indices[LT.indptr[i]:LT.indptr[i + 1]] for i in sample]))
    rows = np.repeat(need, np.diff(L.indptr)[need])
    cols = np.concatenate([L.indices[L.indptr[k]:L.indptr[k + 1]] for k in need])
    ev = (cx.xyz[cx.edges[:, 1]] - cx.xyz[cx.edges[:, 0]])[ie]
    f = Lr.features(A, Me, Sm, tau, ev, rows, cols)
    o, _ = Lr.mlp_forward(w32, f)
    G, gref = Lr.factor(o, rows, cols, A.diagonal(), n)
    Gm, bound = factor_model(w32, f, rows, cols, A.diagonal())
    dG = sp.csr_matrix((np.abs(Gm - gref) + bound + 2.0 ** -8 * (np.abs(Gm) + bound), (rows, cols)), shape=(n, n))
    aG, ar = abs(G), np.abs(r)
    zo = (G.T @ (G @ r))[sample]
    tol = (aG.T @ (dG @ ar) + dG.T @ (aG @ ar) + dG.T @ (dG @ ar) + 1e-13 * (aG.T @ (aG @ ar)))[sample]
    assert (np.abs(z[sample] - zo) <= tol).all()
    gr, gc, gv = ctx.precond_factor()
    Gb = sp.csr_matrix((_bf16(gv), (gr, gc)), shape=(n, n))
    zb = Gb.T @ (Gb @ r)
    aGb = abs(Gb)
    assert (np.abs(z - zb) <= 64 * np.finfo(float).eps * (aGb.T @ (aGb @ ar))).all()
    ctx.close()


def test_plasma64_order_independent(plasma64):
    """The 64^3 / 16M cycle from the particles in their generated order and in a shuffled one,
    with the same trained preconditioner (saved from the first context, loaded into the second):
    three full steps (a sort in between) give bit-identical fields, deposits and particles by id."""
    import paper_2103_06737_amd as qh
    cfg, mesh, parts, cx, op, po = plasma64
    x, v, tet = parts["e"]
    perm = np.random.default_rng(32).permutation(tet.size)
    blob, runs = None, []
    for order in (None, perm):
        ctx = gpu_context(mesh, cfg["dt"], weight=cfg["weight"])
        ctx.fields_init_synthetic(qi.white(cx.Ne, 0, 3), qi.white(cx.Ne, 0, 5), cfg["sigma_e"], cfg["bz"],
                                  cfg["sigma_b"])
        sid = ctx.species_add(-qi.QE / qi.ME, -1)
        if order is None:
            ctx.particles_upload(sid, x, v, tet)
        else:
            ctx.particles_upload(sid, x[order], v[order], tet[order])
        ctx.charge_background(1)
        if blob is None:
            ctx.precond_train(steps=30, lr=3e-3, seed=1, validate_every=0)
            blob = ctx.precond_save()
        else:
            ctx.precond_load(blob)
        params = ctx.step_params(field_mode=qh.FIELDS_SOLVE, precond=qh.PC_LEARNED, sort_every=2)
        st = ctx.pic_step(params, 3)
        assert all(s["fallbacks"] == 0 for s in st)
        xs, vs, ts = ctx.particles_download(sid)
        if order is not None:
            back = np.empty_like(order)
            back[order] = np.arange(order.size)
            xs, vs, ts = xs[back], vs[back], ts[back]
        runs.append(ctx.fields_download() + ctx.deposits_download() + (xs, vs, ts))
        ctx.close()
    for a, ref in zip(runs[1], runs[0]):
        assert np.array_equal(a, ref)


def test_plasma64_field_energy(plasma64):
    """Field energy on the 64^3 mesh (Sec. VI.A.1): the uniform B_z of the plasma workload has
    the closed form B_z^2 V / (2 mu0) (its fluxes are rounded to u_b, a relative 1e-12); random
    fields agree with the oracle's Hodge quadratic forms within a rounding bound; and three
    source-free steps (Jacobi PCG to 1e-12, no Gauss-law solve) keep the sum."""
    import paper_2103_06737_amd as qh
    cfg, mesh, parts, cx, op, po = plasma64
    ctx = gpu_context(mesh, cfg["dt"], weight=cfg["weight"], u_b=U_B)
    ctx.fields_init_synthetic(qi.white(cx.Ne, 0, 3), qi.white(cx.Ne, 0, 5), 0.0, cfg["bz"], 0.0)
    we, wm = ctx.fields_energy()
    vol = np.prod(mesh.xyz.max(axis=0) - mesh.xyz.min(axis=0))
    assert we == 0.0
    assert abs(wm - cfg["bz"] ** 2 * vol / (2 * qi.MU0)) <= 1e-9 * wm
    # E and cB of one size, so that the exchange between the two parts is visible in the sum
    ctx.fields_init_synthetic(qi.white(cx.Ne, 1, 3), qi.white(cx.Ne, 1, 5), 3e5, 0.0, 1e-3)
    e, b = ctx.fields_download()
    we, wm = ctx.fields_energy()
    assert 0.1 < we / wm < 10
    br = b * U_B
    tiny = 64 * np.finfo(float).eps
    assert abs(we - 0.5 * e @ (op.Meps @ e)) <= tiny * 0.5 * np.abs(e) @ (abs(op.Meps) @ np.abs(e))
    assert abs(wm - 0.5 * br @ (op.Mmu @ br)) <= tiny * 0.5 * np.abs(br) @ (abs(op.Mmu) @ np.abs(br))
    w0 = we + wm
    params = ctx.step_params(field_mode=qh.FIELDS_SOLVE, gauss=0, tol_edge=1e-12, max_it_edge=4000)
    for _ in range(3):
        st = ctx.pic_step(params)[0]
        we1, wm1 = ctx.fields_energy()
        assert abs(we1 + wm1 - w0) <= 1e-10 * w0, st
    assert abs(we1 - we) > 1e-4 * w0  # energy did pass between the electric and magnetic parts
    ctx.close()


def test_plasma64_plane_wave_natural_boundary(plasma64):
    """Natural walls and a plane-wave pulse (300 MHz, 150 MHz bandwidth, its peak passing x = 0 at
    t = 0) on the 64^3 / 16M workload, unmagnetised (natural walls carry no surface current to
    hold a static B), with the learned preconditioner, as the benchmark's plane-wave run
    launches it. One step, piece by piece: the edge right-hand side is the
    oracle's source-free one plus a boundary term that vanishes off the wall edges and equals the
    oracle's on 256 sampled wall edges (integrated over their wall faces only); the solution's
    residual; the Gauss law with the charge and the normal flux G^T of that term; the integer
    Faraday update bit for bit."""
    import copy
    import paper_2103_06737_amd as qh
    from oracle.field import FieldOracle, PlaneWave
    cfg, mesh, parts, cx, op, po = plasma64
    cxn = copy.copy(cx)
    cxn.neumann = True
    dt, weight = cfg["dt"], cfg["weight"]
    u_q = qi.QE * weight * 2.0 ** -40
    ctx = qh.Context(0)
    ctx.set_boundary(qh.BC_NEUMANN)
    ctx.mesh_upload(mesh.xyz, mesh.tets)
    ctx.set_physics(qi.EPS0, qi.MU0, dt, u_q, U_B)
    ctx.fields_init_synthetic(qi.white(cx.Ne, 0, 3), qi.white(cx.Ne, 0, 5), cfg["sigma_e"], 0.0,
                              cfg["sigma_b"])
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    x, v, tet = parts["e"]
    ctx.particles_upload(sid, x, v, tet)
    ctx.charge_background(1)
    f0, bw, t0 = 300e6, 150e6, 0.0
    E0 = 1e3 / (2 * np.pi * f0)    # E_inc = E0 s', s' peaks near 2 pi f0: about 1 kV/m
    ctx.set_plane_wave(E0, f0, bw, t0)
    ctx.precond_train(steps=60, lr=3e-3, seed=1, validate_every=0)
    e0, b0 = ctx.fields_download()
    _, Q0 = ctx.deposits_download()
    params = ctx.step_params(field_mode=qh.FIELDS_SOLVE, precond=qh.PC_LEARNED, sort_every=20, verify=1)
    st = ctx.pic_step(params)[0]
    assert st["continuity_bad"] == 0 and st["divb_bad"] == 0 and st["lost"] == 0
    assert st["fallbacks"] == 0 and st["edge_res"] <= 1e-8 and st["gauss_res"] <= 1e-8
    g, Q1 = ctx.deposits_download()
    e1, b1 = ctx.fields_download()
    rhs, sol = ctx.edge_system_download()
    ctx.close()

    fo = FieldOracle(cxn, op, dt)
    b_real, g_real = b0.astype(np.float64) * U_B, g.astype(np.float64) * u_q
    h_dev = rhs - fo.rhs(e0, b_real, g_real)
    terms = abs(fo.Bm) @ np.abs(e0) + dt * (abs(op.CtMmu) @ np.abs(b_real)) + np.abs(g_real)
    tol = 64 * np.finfo(float).eps
    off = ~cx.wall_edge
    assert (np.abs(h_dev[off]) <= tol * terms[off]).all()
    sample = np.random.default_rng(5).choice(np.flatnonzero(cx.wall_edge), 256, replace=False)
    faces = np.intersect1d(cx.C[:, sample].nonzero()[0], np.flatnonzero(cx.wall_face))
    pw = PlaneWave(cxn, op, E0, f0, bw, t0, faces=faces)
    hs = 0.5 * dt * (pw.h(0.0) + pw.h(dt))
    # rounding scale of the source: s' = env (-(u/sig^2) cos(om u) - om sin(om u)) cancels near its
    # zeros, and the rounding of the arguments om u and u^2/(2 sig^2) moves cos, sin and env by
    # about eps times the argument, so each point counts with the size of both terms times the
    # arguments' condition
    habs = np.zeros(cx.Ne)
    om = 2 * np.pi * f0
    for t in (0.0, dt):
        u = t - pw.xq / pw.c - pw.t0
        y = u * u / (2 * pw.sig ** 2)
        part = np.exp(-y) * (np.abs(u) / pw.sig ** 2 + om) * (1.0 + np.abs(om * u) + y)
        np.add.at(habs, pw.edges, 0.5 * dt * np.abs(pw.coef) * part * pw.E0 / pw.eta)
    assert np.abs(hs[sample]).max() > 1e6 * tol * terms[sample].max()    # the source is not lost in rounding
    ratio = np.abs(h_dev[sample] - hs[sample]) / (tol * (terms[sample] + habs[sample]))
    assert ratio.max() <= 1.0, (ratio.max(), np.abs(h_dev[sample] - hs[sample]).max())
    assert np.linalg.norm(fo.A @ sol - rhs) <= 1.001e-8 * np.linalg.norm(rhs)
    rho = u_q * (Q0 - Q1).astype(np.float64) + fo.Gf.T @ h_dev    # Q_bg = Q0
    assert fo.gauss_error(e1, rho) <= 1.01e-8
    u = np.rint((0.5 * dt / U_B) * (e1 + e0)).astype(np.int64)
    assert np.array_equal(b1, b0 - cx.C @ u)
    assert np.array_equal(cx.D @ b1, cx.D @ b0)


def test_beam32_200_steps():
    """1M-electron beam in frozen random fields, 200 steps: continuity and D b every step on the
    device, FP32 positions within 1e-5 of the box size of the FP64 oracle's after 200 steps.

    Tie-consistent replay: E jumps across faces, so a particle that the two arithmetics place on
    different sides of a face would see different fields from then on. After each step the
    oracle adopts the GPU's tet when the gap is explained by the FP32/FP64 position difference
    d of that particle: its own point lies inside the GPU's tet up to |grad lambda| d (twice,
    plus 1e-6 for the FP32 point itself). Likewise at the walls (the planes of the unit cube): a
    particle that ends the step within 1e-5 of a wall may be reflected by one arithmetic and
    not (yet) by the other; the oracle then takes the GPU's sign of that velocity component."""
    cfg = qi.CONFIGS["beam32"]
    mesh = qi.make_mesh(cfg)
    cx, op, po = oracle_setup(mesh)
    e, b = oracle_fields(cx, cfg, U_B)
    x, v, tet = qi.make_particles(mesh, cfg)["e"]
    assert tet.size == 1_000_000
    ctx = gpu_context(mesh, cfg["dt"])
    ctx.fields_upload(e, b)
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    ctx.particles_upload(sid, x, v, tet)
    xo, vo, to = x.astype(np.float64), v.astype(np.float64), tet.astype(np.int64)
    params = ctx.step_params(sort_every=20, verify=1)
    crossings = 0
    for _ in range(200):
        st = ctx.pic_step(params)[0]
        assert st["continuity_bad"] == 0 and st["divb_bad"] == 0 and st["lost"] == 0
        crossings += st["crossings"]
        out = po.push(e, b * U_B, xo, vo, to, -qi.QE / qi.ME, cfg["dt"], -1)
        xo, vo, to = out["x"], out["v"], out["tet"]
        xg, vg, tg = ctx.particles_download(sid)
        near_wall = np.minimum(xo, 1.0 - xo) <= 1e-5
        flip = near_wall & (np.sign(vg) != np.sign(vo)) & (np.abs(np.abs(vg) - np.abs(vo)) <= 1e-3 * np.abs(vo))
        vo[flip] = -vo[flip]
        diff = np.flatnonzero(tg != to)
        if diff.size:
            M = op.Minv[tg[diff]]
            lam = M[:, :, 0] + np.einsum("ijk,ik->ij", M[:, :, 1:], xo[diff])
            grad = np.linalg.norm(M[:, :, 1:], axis=2).max(axis=1)
            band = 2.0 * grad * np.abs(xg[diff] - xo[diff]).max(axis=1) + 1e-6
            tie = lam.min(axis=1) >= -band
            to[diff[tie]] = tg[diff[tie]]
    assert crossings > 1_000_000
    xg, vg, tg = ctx.particles_download(sid)
    assert np.array_equal(tg, to)
    assert np.abs(xg - xo).max() <= 1e-5
    record("beam32_200_steps", dict(x_abs_m=err_stats(np.abs(xg - xo).max(axis=1)),
                                    v_rel=err_stats(np.abs(vg - vo).max(axis=1) / np.abs(vo).max())))


def test_graded96_two_species():
    """96^3 mesh graded toward z = 0 (5.3M tets), electrons and ions (2M each here, the full
    workload's mesh and species mix), full cycle with Jacobi and then the learned
    preconditioner: continuity (on the device every step, and on the host), D b, residuals,
    and fewer edge iterations with the trained network."""
    import paper_2103_06737_amd as qh
    from oracle.complex_ import Complex
    cfg = qi.CONFIGS["graded96"]
    mesh = qi.make_mesh(cfg)
    n_e = 2_000_000
    parts = qi.make_particles(mesh, cfg, n_e=n_e)
    weight = cfg["weight"] * cfg["n_e"] / n_e
    ctx = gpu_context(mesh, cfg["dt"], weight=weight)
    mi = ctx.mesh_info()
    assert mi.n_tets == 6 * 96 ** 3
    # rows here span two z-layers of 97^2 nodes (~129 K columns), yet every tile's columns fit
    # three 2^14-column windows: 16-bit columns throughout
    assert mi.nnz_edge_c16 == mi.nnz_edge
    ctx.fields_init_synthetic(qi.white(mi.n_edges, 0, 3), qi.white(mi.n_edges, 0, 5), cfg["sigma_e"], cfg["bz"],
                              cfg["sigma_b"])
    for name, (x, v, tet) in parts.items():
        qm, z = (-qi.QE / qi.ME, -1) if name == "e" else (qi.QE / qi.MI, 1)
        ctx.particles_upload(ctx.species_add(qm, z), x, v, tet)
    ctx.charge_background(1)
    cx = Complex(mesh.xyz, mesh.tets)
    # one step of both species against the oracle's push of 4096 sampled particles of each, with
    # the species' own q/m and charge number, through the same start fields
    from oracle.particles import ParticleOracle
    from oracle.whitney import barycentric
    po = ParticleOracle(cx, barycentric(cx)[0])
    e0, b0 = ctx.fields_download()
    start = {k: ctx.particles_download(s) for k, s in enumerate((0, 1))}
    ctx.pic_step(ctx.step_params(verify=1))
    rng = np.random.default_rng(96)
    for k, (qm, z) in enumerate(((-qi.QE / qi.ME, -1), (qi.QE / qi.MI, 1))):
        x, v, tet = start[k]
        xg, vg, tg = ctx.particles_download(k)
        idx = rng.choice(tet.size, 4096, replace=False)
        orc = po.push(e0, b0 * U_B, x[idx], v[idx], tet[idx], qm, cfg["dt"], z)
        same = tg[idx] == orc["tet"]
        assert same.mean() > 0.999, k
        assert np.abs(xg[idx] - orc["x"]).max(axis=1)[same].max() < 1e-5, k
        assert (np.abs(vg[idx] - orc["v"]).max(axis=1)[same] / np.abs(orc["v"]).max()).max() < 1e-5, k
    del start, po
    iters = {}
    for pc in (qh.PC_JACOBI, qh.PC_LEARNED):
        if pc == qh.PC_LEARNED:
            ctx.precond_train(steps=60, lr=3e-3, seed=1, validate_every=0)
        params = ctx.step_params(field_mode=qh.FIELDS_SOLVE, precond=pc, sort_every=20, verify=1)
        for _ in range(2):
            _, Q0 = ctx.deposits_download()
            st = ctx.pic_step(params)[0]
            g, Q1 = ctx.deposits_download()
            assert st["continuity_bad"] == 0 and st["divb_bad"] == 0 and st["lost"] == 0
            assert st["fallbacks"] == 0 and st["edge_res"] <= 1e-8 and st["gauss_res"] <= 1e-8
            assert np.array_equal(cx.G.T @ g, Q1 - Q0)
        iters[pc] = st["edge_iters"]
    assert iters[qh.PC_LEARNED] < 0.75 * iters[qh.PC_JACOBI]


def test_graded96_full_run():
    """The graded workload at its full size and length: 96^3 graded mesh, 32M electrons and 32M
    ions, learned preconditioner with the mixed-precision edge solve (the benchmark's), 200 steps
    with a re-sort every 20, every invariant checked on the device at every step; total charge and
    D b on the host at the end."""
    import paper_2103_06737_amd as qh
    cfg = qi.CONFIGS["graded96"]
    mesh = qi.make_mesh(cfg)
    parts = qi.make_particles(mesh, cfg)
    ctx = gpu_context(mesh, cfg["dt"], weight=cfg["weight"])
    mi = ctx.mesh_info()
    ctx.fields_init_synthetic(qi.white(mi.n_edges, 0, 3), qi.white(mi.n_edges, 0, 5), cfg["sigma_e"], cfg["bz"],
                              cfg["sigma_b"])
    sids = {}
    for name, (x, v, tet) in parts.items():
        qm, z = (-qi.QE / qi.ME, -1) if name == "e" else (qi.QE / qi.MI, 1)
        sids[name] = ctx.species_add(qm, z)
        ctx.particles_upload(sids[name], x, v, tet)
    del parts
    ctx.charge_background(1)
    ctx.precond_train(steps=60, lr=3e-3, seed=1, validate_every=0)
    _, b0 = ctx.fields_download()
    _, Q0 = ctx.deposits_download()
    params = ctx.step_params(field_mode=qh.FIELDS_SOLVE, precond=qh.PC_LEARNED, sort_every=cfg["sort_every"],
                             verify=1, solver=qh.SOLVER_MIXED)
    stats = []
    for _ in range(4):
        stats += ctx.pic_step(params, cfg["steps"] // 4)
        print(f"graded96: {len(stats)} steps, edge iterations {stats[-1]['edge_iters']}", flush=True)
    assert len(stats) == 200
    for k, st in enumerate(stats):
        assert st["continuity_bad"] == 0 and st["divb_bad"] == 0 and st["lost"] == 0, (k, st)
        assert st["fallbacks"] == 0 and st["edge_res"] <= 1e-8 and st["gauss_res"] <= 1e-8, (k, st)
    _, Q1 = ctx.deposits_download()
    _, b1 = ctx.fields_download()
    assert Q1.sum() == Q0.sum()
    from oracle.complex_ import Complex
    cx = Complex(mesh.xyz, mesh.tets)
    assert np.array_equal(cx.D @ b1, cx.D @ b0)
    assert all(ctx.particles_count(s) == 32_000_000 for s in sids.values())
    ctx.close()
