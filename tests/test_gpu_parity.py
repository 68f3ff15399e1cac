"""HIP path vs the FP64 oracle, through the C ABI (needs an MI355X).

Bars: integer deposits bit-exact; continuity G^T g = Q^{n+1} - Q^n and D b = const bit-exact on
the GPU every step; FP32 positions within 1e-5 of the box size after 100 steps under
tie-consistent replay; field solve residuals <= 1e-8 recomputed in FP64; the GPU field update
equals the oracle's applied to the same state and deposits to the solver tolerance.
"""
import numpy as np
import pytest

import qh_inputs as qi

from .gpu_setup import (GATHER_REL, PUSH_V_REL, PUSH_X_ABS, S, chained_segments, err_stats, gpu_context,
                        node_charge, oracle_fields,
                        oracle_setup, record)

pytestmark = pytest.mark.gpu

U_B = 2.0 ** -56


@pytest.fixture(scope="module")
def jitter4():
    cfg = qi.CONFIGS["jitter4"]
    mesh = qi.make_mesh(cfg)
    cx, op, po = oracle_setup(mesh)
    e, b = oracle_fields(cx, cfg, U_B)
    parts = qi.make_particles(mesh, cfg)
    return cfg, mesh, cx, op, po, e, b, parts


def test_deposit_lists_bit_exact(jitter4):
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    ctx = gpu_context(mesh, cfg["dt"])
    for seed in range(3):
        st, l0, l1, sz, pt, pl, pz = chained_segments(cx, 3000, seed)
        g_gpu, Q_gpu = ctx.deposit(st, l0, l1, sz, pt, pl, pz)
        g_orc, Q_orc = po.deposit_list(st, l0, l1, sz, pt, pl, pz)
        assert np.array_equal(g_gpu, g_orc)
        assert np.array_equal(Q_gpu, Q_orc)
    # empty lists
    g0, Q0 = ctx.deposit(np.zeros(0), np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0),
                         np.zeros(0), np.zeros((0, 4)), np.zeros(0))
    assert not g0.any() and not Q0.any()


def test_synthetic_fields_match_oracle(jitter4):
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    ctx = gpu_context(mesh, cfg["dt"])
    ctx.fields_init_synthetic(qi.white(cx.Ne, 0, 3), qi.white(cx.Ne, 0, 5), 1e3, 0.1, 1e-3)
    eg, bg = ctx.fields_download()
    from oracle.field import init_fields
    eo, bo = init_fields(cx, qi.white(cx.Ne, 0, 3), qi.white(cx.Ne, 0, 5), 1e3, 0.1, 1e-3, U_B)
    assert np.allclose(eg, eo, rtol=1e-14, atol=0)
    assert np.abs(bg - bo).max() <= 3
    assert not (cx.D @ bg).any()


def _stress_step(jitter4, n=1000):
    """One step with displacements of order a cell: many crossings and wall hits."""
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    dt = 2e-9
    ctx = gpu_context(mesh, dt)
    ctx.fields_upload(e, b)
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    x, v, tet = parts["e"]
    v = (v * 40.0).astype(np.float32)
    ctx.particles_upload(sid, x[:n], v[:n], tet[:n])
    _, Q0 = ctx.deposits_download()
    ctx.capture_segments(64 * n)
    st = ctx.pic_step(ctx.step_params(verify=1))[0]
    xg, vg, tg = ctx.particles_download(sid)
    g, Q1 = ctx.deposits_download()
    nseg, seg = ctx.segments_download()
    orc = po.push(e, b * U_B, x[:n], v[:n], tet[:n], -qi.QE / qi.ME, dt, -1)
    return dict(ctx=ctx, st=st, x0=x[:n], v0=v[:n], t0=tet[:n], xg=xg, vg=vg, tg=tg, g=g, Q0=Q0, Q1=Q1,
                nseg=nseg, seg=seg, orc=orc)


def test_one_step_integer_path_bit_exact(jitter4):
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    r = _stress_step(jitter4)
    st = r["st"]
    assert st["crossings"] > 200 and st["wall_hits"] > 10 and st["lost"] == 0
    assert st["continuity_bad"] == 0
    # continuity, bit for bit
    assert np.array_equal(cx.G.T @ r["g"], r["Q1"] - r["Q0"])
    # Q0 equals the oracle's W0 charge of the same FP32 start points (FP32 lambda in a tie
    # band can differ by one unit; all others equal)
    Qo = node_charge(po, cx, r["x0"], r["t0"], -1)
    per_node = np.bincount(cx.tets[r["t0"]].ravel(), minlength=cx.Nn)
    assert (np.abs(r["Q0"] - Qo) <= 4 * S * per_node).all()
    # the GPU's own pieces, re-deposited by the oracle, reproduce its g and Q bit for bit
    seg = r["seg"]
    assert r["nseg"] == seg["tet"].size
    g_re, _ = po.deposit_list(seg["tet"], seg["lam0"], seg["lam1"], -np.ones(seg["tet"].size),
                              np.zeros(0), np.zeros((0, 4)), np.zeros(0))
    assert np.array_equal(g_re, r["g"])
    order = np.lexsort((seg["seq"], seg["pid"]))
    pid, seq = seg["pid"][order], seg["seq"][order]
    last = np.r_[pid[1:] != pid[:-1], True]
    _, Q_re = po.deposit_list(np.zeros(0), np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0),
                              seg["tet"][order][last], seg["lam1"][order][last], -np.ones(last.sum()))
    assert np.array_equal(Q_re, r["Q1"])
    # every piece's coordinates sum to 2^20; chained pieces share their face point
    assert (seg["lam0"].sum(1) == S).all() and (seg["lam1"].sum(1) == S).all()
    assert np.unique(pid).size == r["x0"].shape[0]


def test_one_step_fp32_vs_fp64(jitter4):
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    r = _stress_step(jitter4)
    orc = r["orc"]
    same = r["tg"] == orc["tet"]
    assert same.mean() > 0.99
    dx = np.abs(r["xg"] - orc["x"]).max(axis=1)
    assert dx[same].max() <= PUSH_X_ABS
    dv = np.abs(r["vg"] - orc["v"]).max(axis=1) / np.abs(orc["v"]).max()
    assert dv[same].max() <= PUSH_V_REL
    # a different final tet only inside the tie band
    for i in np.flatnonzero(~same):
        lam = op.Minv[r["tg"][i], :, 0] + op.Minv[r["tg"][i], :, 1:] @ orc["x"][i]
        assert lam.min() > -1e-5
    # piece end points agree with FP64 barycentrics to a few units of 2^-20
    seg = r["seg"]
    order = np.lexsort((seg["seq"], seg["pid"]))
    first = np.r_[True, seg["pid"][order][1:] != seg["pid"][order][:-1]]
    i0 = order[first]
    lam0 = np.einsum("pij,pj->pi", op.Minv[seg["tet"][i0], :, 1:], r["x0"][seg["pid"][i0]].astype(np.float64)) \
        + op.Minv[seg["tet"][i0], :, 0]
    dlam = np.abs(seg["lam0"][i0] - np.clip(lam0, 0, 1) * S)
    # FP32 barycentrics of a start point err by about |grad lambda| |x| 2^-24 (a unit of 2^-20 or
    # less here); rounding adds half a unit per coordinate and the largest coordinate takes the
    # other three's remainder: at most 4 units
    assert dlam.max() <= 4
    # the FP32 gather (per-tet records read through the probe) against FP64 at the start points
    Ep, Bp = r["ctx"].probe_fields(r["x0"].astype(np.float64), r["t0"])
    Eo, Bo = po.gather(e, b * U_B, r["x0"].astype(np.float64), r["t0"])
    assert np.abs(Ep - Eo).max() <= GATHER_REL * np.abs(Eo).max()
    assert np.abs(Bp - Bo).max() <= GATHER_REL * np.abs(Bo).max()
    record("jitter4_one_step", dict(
        E_rel=err_stats(np.abs(Ep - Eo).max(axis=1) / np.abs(Eo).max()),
        B_rel=err_stats(np.abs(Bp - Bo).max(axis=1) / np.abs(Bo).max()),
        x_abs_m=err_stats(dx[same]), v_rel=err_stats(dv[same]), lambda_units=err_stats(dlam),
        same_tet=float(same.mean())))


def test_two_species_vs_oracle(jitter4):
    """Electrons (q/m = -e/m_e, z = -1) and ions (q/m = +e/(1836 m_e), z = +1, the graded
    workload's second species) in one context: after one step each species' positions and
    velocities against the oracle's push with its own q/m and charge number (1e-5), both
    species' pieces re-deposited by the oracle with their signs give g and Q bit for bit, and
    continuity holds on the host; then 20 steps under tie-consistent replay per species."""
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    dt = 2e-9
    xe, ve, te = parts["e"]
    ve = (ve * 20.0).astype(np.float32)
    rng = np.random.default_rng(41)
    # quiet start: each ion on an electron's position, thermal speeds raised so ions cross tets
    xi, ti = xe.copy(), te.copy()
    vi = rng.normal(0.0, 3e7, xe.shape).astype(np.float32)
    sp = {"e": (-qi.QE / qi.ME, -1, xe, ve, te), "i": (qi.QE / qi.MI, 1, xi, vi, ti)}
    ctx = gpu_context(mesh, dt)
    ctx.fields_upload(e, b)
    sid = {k: ctx.species_add(qm, z) for k, (qm, z, *_r) in sp.items()}
    for k, (qm, z, x, v, t) in sp.items():
        ctx.particles_upload(sid[k], x, v, t)
    _, Q0 = ctx.deposits_download()
    assert not Q0.any()                                    # quiet start: neutral node by node
    ctx.capture_segments(64 * 2 * xe.shape[0])
    st = ctx.pic_step(ctx.step_params(verify=1))[0]
    assert st["continuity_bad"] == 0 and st["lost"] == 0 and st["crossings"] > 500
    g, Q1 = ctx.deposits_download()
    assert np.array_equal(cx.G.T @ g, Q1 - Q0)
    for k, (qm, z, x, v, t) in sp.items():
        xg, vg, tg = ctx.particles_download(sid[k])
        orc = po.push(e, b * U_B, x, v, t, qm, dt, z)
        same = tg == orc["tet"]
        assert same.mean() > 0.99, k
        assert np.abs(xg - orc["x"]).max(axis=1)[same].max() < 1e-5, k
        assert (np.abs(vg - orc["v"]).max(axis=1)[same] / np.abs(orc["v"]).max()).max() < 1e-5, k
    nseg, seg = ctx.segments_download()
    assert nseg == seg["tet"].size
    zs = np.where(seg["species"] == sid["e"], -1, 1)
    g_re, _ = po.deposit_list(seg["tet"], seg["lam0"], seg["lam1"], zs, np.zeros(0), np.zeros((0, 4)), np.zeros(0))
    assert np.array_equal(g_re, g)
    order = np.lexsort((seg["seq"], seg["pid"], seg["species"]))
    key = seg["species"][order].astype(np.int64) * (1 << 32) + seg["pid"][order]
    last = np.r_[key[1:] != key[:-1], True]
    assert last.sum() == 2 * xe.shape[0]
    _, Q_re = po.deposit_list(np.zeros(0), np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0),
                              seg["tet"][order][last], seg["lam1"][order][last], zs[order][last])
    assert np.array_equal(Q_re, Q1)
    # 20 more steps, each species replayed by the oracle with its own q/m and z
    state = {k: [ctx.particles_download(sid[k])[j].astype(np.float64 if j < 2 else np.int64) for j in range(3)]
             for k in sp}
    for _ in range(20):
        st = ctx.pic_step(ctx.step_params(verify=1))[0]
        assert st["continuity_bad"] == 0 and st["lost"] == 0
        for k, (qm, z, *_r) in sp.items():
            xo, vo, to = state[k]
            out = po.push(e, b * U_B, xo, vo, to, qm, dt, z)
            xo, vo, to = out["x"], out["v"], out["tet"]
            xg, _, tg = ctx.particles_download(sid[k])
            for i in np.flatnonzero(tg != to):
                lam = op.Minv[tg[i], :, 0] + op.Minv[tg[i], :, 1:] @ xo[i]
                if lam.min() >= -1e-5:
                    to[i] = tg[i]
            state[k] = [xo, vo, to]
    for k in sp:
        xg, vg, tg = ctx.particles_download(sid[k])
        assert np.array_equal(tg, state[k][2]), k
        assert np.abs(xg - state[k][0]).max() <= 1e-5, k


def test_positions_100_steps_tie_consistent(jitter4):
    """FP32 positions within 1e-5 of the box size after 100 steps; the oracle adopts the GPU's
    tet whenever its own point lies within 1e-5 of it (tie band), and counts those events."""
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    ctx = gpu_context(mesh, cfg["dt"])
    ctx.fields_upload(e, b)
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    x, v, tet = parts["e"]
    ctx.particles_upload(sid, x, v, tet)
    xo, vo, to = x.astype(np.float64), v.astype(np.float64), tet.astype(np.int64)
    params = ctx.step_params(verify=1)
    ties = 0
    for _ in range(100):
        st = ctx.pic_step(params)[0]
        assert st["continuity_bad"] == 0
        out = po.push(e, b * U_B, xo, vo, to, -qi.QE / qi.ME, cfg["dt"], -1)
        xo, vo, to = out["x"], out["v"], out["tet"]
        _, _, tg = ctx.particles_download(sid)
        diff = np.flatnonzero(tg != to)
        for i in diff:
            lam = op.Minv[tg[i], :, 0] + op.Minv[tg[i], :, 1:] @ xo[i]
            if lam.min() >= -1e-5:
                to[i] = tg[i]
                ties += 1
    xg, vg, tg = ctx.particles_download(sid)
    assert np.abs(xg - xo).max() <= 1e-5
    assert np.array_equal(tg, to)
    record("jitter4_100_steps", dict(x_abs_m=err_stats(np.abs(xg - xo).max(axis=1)),
                                     v_rel=err_stats(np.abs(vg - vo).max(axis=1) / np.abs(vo).max()), ties=ties))


@pytest.mark.parametrize("solver", ["fp64", "mixed"])
def test_full_cycle_field_update_matches_oracle(jitter4, solver):
    """Each GPU field update equals the oracle's applied to the same state and deposits, with the
    FP64 edge solve and with the mixed-precision one (FP32 PCG with FP64 reliable updates,
    stopping on the same FP64 residual); halfway the time step changes, so A (and its FP32 copy)
    is formed again."""
    import paper_2103_06737_amd as qh
    from oracle.field import FieldOracle
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    dt = 2e-10
    ctx = gpu_context(mesh, dt)
    ctx.fields_upload(e, b)
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    x, v, tet = parts["e"]
    ctx.particles_upload(sid, x, (v * 20).astype(np.float32), tet)
    fo = FieldOracle(cx, op, dt)
    u_q = qi.QE * 2.0 ** -40
    params = ctx.step_params(field_mode=1, verify=1, tol_edge=1e-10, tol_node=1e-10,
                             solver=qh.SOLVER_MIXED if solver == "mixed" else qh.SOLVER_FP64)
    Qbg = np.zeros(cx.Nn, np.int64)
    for k in range(8):
        if k == 4:
            dt = 3e-10
            ctx.set_physics(qi.EPS0, qi.MU0, dt, u_q, U_B)
            fo = FieldOracle(cx, op, dt)
        e_n, b_n = ctx.fields_download()
        st = ctx.pic_step(params)[0]
        assert st["continuity_bad"] == 0 and st["divb_bad"] == 0
        assert st["edge_res"] <= 1e-10 * 1.0001 and st["fallbacks"] == 0
        assert (st["edge_refinements"] >= 1) == (solver == "mixed")
        assert st["gauss_res"] <= 1e-9
        e_g, b_g = ctx.fields_download()
        g, Q = ctx.deposits_download()
        e_o, b_o, info = fo.step(e_n, b_n, U_B, g, u_q, Q, Qbg, tol=1e-13, tol_n=1e-13)
        assert np.linalg.norm(e_g - e_o) <= 1e-8 * np.linalg.norm(e_o)
        assert np.abs(b_g - b_o).max() <= 2 + 1e-9 * np.abs(b_o).max()
        assert not (cx.D @ b_g).any()


@pytest.mark.parametrize("solver", ["fp64", "mixed"])
def test_wave_field_update_matches_oracle(jitter4, solver):
    """Field updates of the wave-equation mode (eq. wave_cont): the first step (no history) is the
    trapezoidal update, every later one equals the oracle's wave update applied to the same
    e^n, e^{n-1}, b^n and step currents; with the FP64 edge solve and the mixed-precision one."""
    import paper_2103_06737_amd as qh
    from oracle.field import FieldOracle, WaveOracle
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    dt = 2e-10
    ctx = gpu_context(mesh, dt)
    ctx.fields_upload(e, b)
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    x, v, tet = parts["e"]
    ctx.particles_upload(sid, x, (v * 20).astype(np.float32), tet)
    fo, wo = FieldOracle(cx, op, dt), WaveOracle(cx, op, dt)
    u_q = qi.QE * 2.0 ** -40
    params = ctx.step_params(field_mode=qh.FIELDS_WAVE, verify=1, tol_edge=1e-10, tol_node=1e-10,
                             solver=qh.SOLVER_MIXED if solver == "mixed" else qh.SOLVER_FP64)
    Qbg = np.zeros(cx.Nn, np.int64)
    e_prev = g_prev = None
    for k in range(8):
        e_n, b_n = ctx.fields_download()
        st = ctx.pic_step(params)[0]
        assert st["continuity_bad"] == 0 and st["divb_bad"] == 0
        assert st["edge_res"] <= 1e-10 * 1.0001 and st["gauss_res"] <= 1e-9
        assert st["fallbacks"] == 0 and (st["edge_refinements"] >= 1) == (solver == "mixed")
        e_g, b_g = ctx.fields_download()
        g, Q = ctx.deposits_download()
        if k == 0:
            e_o, b_o, _ = fo.step(e_n, b_n, U_B, g, u_q, Q, Qbg, tol=1e-13, tol_n=1e-13)
        else:
            rho = u_q * (Qbg - Q).astype(np.float64)[cx.int_nodes]
            e_o, b_o, _ = wo.wave_step(e_n, e_prev, b_n, U_B, g, g_prev, u_q, rho, tol=1e-13, tol_n=1e-13)
        assert np.linalg.norm(e_g - e_o) <= 1e-8 * np.linalg.norm(e_o)
        assert np.abs(b_g - b_o).max() <= 2 + 1e-9 * np.abs(b_o).max()
        assert not (cx.D @ b_g).any()
        e_prev, g_prev = e_n, g


def test_wave_mode_equals_trapezoidal_source_free(jitter4):
    """Without particles the wave-equation mode and the trapezoidal mode give the same fields
    (Newmark beta = 1/4 on the wave equation is the trapezoidal rule with b eliminated), step
    after step, to the solver tolerance."""
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    dt = 2e-10
    out = {}
    for mode in (qh.FIELDS_SOLVE, qh.FIELDS_WAVE):
        ctx = gpu_context(mesh, dt)
        ctx.fields_upload(e, b)
        ctx.pic_step(ctx.step_params(field_mode=mode, tol_edge=1e-12, tol_node=1e-12), 12)
        out[mode] = ctx.fields_download()
    e_t, b_t = out[qh.FIELDS_SOLVE]
    e_w, b_w = out[qh.FIELDS_WAVE]
    assert np.linalg.norm(e_w - e_t) <= 1e-8 * np.linalg.norm(e_t)
    assert np.abs(b_w - b_t).max() <= 2 + 1e-8 * np.abs(b_t).max()


@pytest.mark.parametrize("solver", ["fp64", "mixed"])
def test_neumann_field_update_matches_oracle(jitter4, solver):
    """Natural boundary (eq. zero_mean_constraint): every edge and node is an unknown and the
    Gauss-law system is singular (constants). The device solves it by CG on the consistent right-
    hand side (a neutral plasma); the oracle on the zero-mean subspace of the paper. e does not
    see the constant, so the field updates agree step by step, with either edge solve."""
    import paper_2103_06737_amd as qh
    from oracle.complex_ import Complex
    from oracle.field import FieldOracle
    from oracle.particles import ParticleOracle
    from oracle.whitney import Operators
    cfg, mesh, _, _, _, _, _, parts = jitter4
    cx = Complex(mesh.xyz, mesh.tets, neumann=True)
    op = Operators(cx, qi.EPS0, qi.MU0)
    e, b = oracle_fields(cx, cfg, U_B)
    assert np.abs(e[cx.wall_edge]).max() > 0
    dt = 2e-10
    ctx = qh.Context(0)
    ctx.set_boundary(qh.BC_NEUMANN)
    ctx.mesh_upload(mesh.xyz, mesh.tets)
    u_q = qi.QE * 2.0 ** -40
    ctx.set_physics(qi.EPS0, qi.MU0, dt, u_q, U_B)
    ctx.fields_upload(e, b)
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    x, v, tet = parts["e"]
    ctx.particles_upload(sid, x, (v * 20).astype(np.float32), tet)
    ctx.charge_background(1)
    _, Q_bg = ctx.deposits_download()
    fo = FieldOracle(cx, op, dt)
    params = ctx.step_params(field_mode=qh.FIELDS_SOLVE, verify=1, tol_edge=1e-10, tol_node=1e-10,
                             solver=qh.SOLVER_MIXED if solver == "mixed" else qh.SOLVER_FP64)
    for k in range(6):
        e_n, b_n = ctx.fields_download()
        st = ctx.pic_step(params)[0]
        assert st["continuity_bad"] == 0 and st["divb_bad"] == 0
        assert st["edge_res"] <= 1e-10 * 1.0001 and st["gauss_res"] <= 1e-9
        assert st["fallbacks"] == 0 and (st["edge_refinements"] >= 1) == (solver == "mixed")
        e_g, b_g = ctx.fields_download()
        g, Q = ctx.deposits_download()
        e_o, b_o, _ = fo.step(e_n, b_n, U_B, g, u_q, Q, Q_bg, tol=1e-13, tol_n=1e-13)
        assert np.linalg.norm(e_g - e_o) <= 1e-8 * np.linalg.norm(e_o)
        assert np.abs(b_g - b_o).max() <= 2 + 1e-9 * np.abs(b_o).max()


@pytest.mark.parametrize("solver", ["fp64", "mixed"])
@pytest.mark.parametrize("mode", ["trapezoidal", "wave"])
def test_plane_wave_through_natural_boundary(mode, solver):
    """Sec. VI.A.2: a resolved plane wave (150 MHz on a 1 m box of 6^3 cells) enters through the
    natural boundary. Every step of the device agrees with the oracle's update from the same
    fields with the same boundary term (step average for the trapezoidal update, central
    difference for the wave update) and the same accumulated boundary flux in the Gauss-law
    target; the field follows the incident wave. Half way the wave is set again (the flux
    already brought in stays); for the last steps it is switched off (no boundary term, the
    flux stays). With the FP64 edge solve and the mixed-precision one."""
    import paper_2103_06737_amd as qh
    from oracle.complex_ import Complex
    from oracle.field import PlaneWave, WaveOracle
    from oracle.whitney import Operators
    mesh = qi.BoxMesh(6, 1.0)
    cx = Complex(mesh.xyz, mesh.tets, neumann=True)
    op = Operators(cx, qi.EPS0, qi.MU0)
    f0, bw, dt = 150e6, 75e6, 0.1e-9
    E0, t0 = 1.0 / (2 * np.pi * f0), 4.0 / (2 * np.pi * bw)
    pw = PlaneWave(cx, op, E0, f0, bw, t0)
    ctx = qh.Context(0)
    ctx.set_boundary(qh.BC_NEUMANN)
    ctx.mesh_upload(mesh.xyz, mesh.tets)
    ctx.set_physics(qi.EPS0, qi.MU0, dt, qi.QE * 2.0 ** -40, U_B)
    ctx.fields_upload(np.zeros(cx.Ne), np.zeros(cx.Nf, np.int64))
    ctx.set_plane_wave(E0, f0, bw, t0)
    fo = WaveOracle(cx, op, dt)
    params = ctx.step_params(field_mode=qh.FIELDS_WAVE if mode == "wave" else qh.FIELDS_SOLVE,
                             verify=1, tol_edge=1e-12, tol_node=1e-12,
                             solver=qh.SOLVER_MIXED if solver == "mixed" else qh.SOLVER_FP64)
    g0 = np.zeros(cx.Ne, np.int64)
    d = np.zeros(cx.Nn)
    e_prev, on, rel = None, True, []
    for k in range(72):
        if k == 30:
            ctx.set_plane_wave(E0, f0, bw, t0)
        if k == 64:
            ctx.set_plane_wave(0.0, f0, bw, t0)
            on = False
        e_n, b_n = ctx.fields_download()
        st = ctx.pic_step(params)[0]
        assert st["divb_bad"] == 0 and st["gauss_res"] <= 1e-9 and st["fallbacks"] == 0
        e_g, b_g = ctx.fields_download()
        h = (lambda t: pw.h(t)) if on else (lambda t: np.zeros(cx.Ne))
        hs = 0.5 * dt * (h(k * dt) + h((k + 1) * dt))
        d += fo.Gint.T @ hs
        if mode == "wave" and k > 0:
            hd = 0.5 * dt * (h((k + 1) * dt) - h((k - 1) * dt))
            e_o, b_o, _ = fo.wave_step(e_n, e_prev, b_n, U_B, g0, g0, 1.0, d, tol=1e-13, tol_n=1e-13, h_diff=hd)
        else:
            e_o, b_o, _ = fo.step_with_rho(e_n, b_n, U_B, g0, 1.0, d, tol=1e-13, tol_n=1e-13, h_sum=hs)
        e_prev = e_n
        assert np.linalg.norm(e_g - e_o) <= 1e-8 * np.linalg.norm(e_o), k
        assert np.abs(b_g - b_o).max() <= 2 + 1e-9 * np.abs(b_o).max(), k
        ref = pw.e_line((k + 1) * dt)
        rel.append(np.linalg.norm(e_g - ref) / np.linalg.norm(ref))
    assert max(rel[40:64]) < 0.15


@pytest.mark.parametrize("bc", ["pec", "neumann"])
def test_fields_decompose_matches_oracle(jitter4, bc):
    """Quasi-Helmholtz split (Sec. III) of a random field: rho_bar = G^T [*eps] e, the potential
    part E_ns = K^{-1} rho_bar (zero W0-weighted mean under natural walls) and E_s = e - G E_ns
    against the oracle's; E_s has no discrete divergence."""
    import paper_2103_06737_amd as qh
    from oracle.complex_ import Complex
    from oracle.field import FieldOracle
    from oracle.whitney import Operators
    cfg, mesh, _, _, _, _, _, _ = jitter4
    cx = Complex(mesh.xyz, mesh.tets, neumann=bc == "neumann")
    op = Operators(cx, qi.EPS0, qi.MU0)
    ctx = qh.Context(0)
    if bc == "neumann":
        ctx.set_boundary(qh.BC_NEUMANN)
    ctx.mesh_upload(mesh.xyz, mesh.tets)
    ctx.set_physics(qi.EPS0, qi.MU0, 1e-10, qi.QE * 2.0 ** -40, U_B)
    e = np.random.default_rng(12).standard_normal(cx.Ne) * 1e3
    if bc == "pec":
        e[cx.wall_edge] = 0.0
    ctx.fields_upload(e, np.zeros(cx.Nf, np.int64))
    e_ns, e_s, rho, st = ctx.fields_decompose(tol=1e-12)
    fo = FieldOracle(cx, op, 1e-10)
    o_ns, o_s, o_rho = fo.decompose(e, tol=1e-14)
    terms = (abs(fo.GtMeps) @ np.abs(e))[cx.int_nodes]
    assert (np.abs(rho[cx.int_nodes] - o_rho) <= 64 * np.finfo(float).eps * terms).all()
    assert np.linalg.norm(e_ns - o_ns) <= 1e-8 * np.linalg.norm(o_ns)
    assert np.linalg.norm(e_s - o_s) <= 1e-8 * np.linalg.norm(o_s)
    div = (fo.GtMeps @ e_s)[cx.int_nodes]
    assert np.linalg.norm(div) <= 1e-10 * np.linalg.norm(terms)
    assert st["iters"] > 0


@pytest.mark.parametrize("bc", ["pec", "neumann"])
def test_field_energy_matches_oracle_and_is_conserved(jitter4, bc):
    """Field energy 1/2 e^T [*eps] e + 1/2 b^T [*mu^-1] b (Sec. VI.A.1). The device evaluates the
    magnetic part per tet from the constant B_T of a flux vector with D b = 0; the oracle takes the
    full quadratic form of its face Hodge matrix, so agreement also pins that identity. Without
    sources the trapezoidal update keeps the sum: with the Gauss-law solve off from a random e,
    and with it on from the solenoidal part E_s (whose correction is then at the tolerance)."""
    import paper_2103_06737_amd as qh
    from oracle.complex_ import Complex
    from oracle.whitney import Operators
    cfg, mesh, _, _, _, _, _, _ = jitter4
    cx = Complex(mesh.xyz, mesh.tets, neumann=bc == "neumann")
    op = Operators(cx, qi.EPS0, qi.MU0)
    from oracle.field import init_fields
    # E and cB of one size, so that the exchange between the two parts is visible in the sum
    e, b = init_fields(cx, qi.white(cx.Ne, 4, 3), qi.white(cx.Ne, 4, 5), 3e5, 0.0, 1e-3, U_B)
    assert not (cx.D @ b).any()
    dt = 2e-10

    def context():
        ctx = qh.Context(0)
        if bc == "neumann":
            ctx.set_boundary(qh.BC_NEUMANN)
        ctx.mesh_upload(mesh.xyz, mesh.tets)
        ctx.set_physics(qi.EPS0, qi.MU0, dt, qi.QE * 2.0 ** -40, U_B)
        return ctx

    def oracle_energy(e, b):
        br = b * U_B
        we, wm = 0.5 * e @ (op.Meps @ e), 0.5 * br @ (op.Mmu @ br)
        bound_e = 64 * np.finfo(float).eps * 0.5 * np.abs(e) @ (abs(op.Meps) @ np.abs(e))
        bound_m = 64 * np.finfo(float).eps * 0.5 * np.abs(br) @ (abs(op.Mmu) @ np.abs(br))
        return we, wm, bound_e, bound_m

    ctx = context()
    ctx.fields_upload(e, b)
    we, wm = ctx.fields_energy()
    o_we, o_wm, be, bm = oracle_energy(e, b)
    assert 0.1 < we / wm < 10
    assert abs(we - o_we) <= be and abs(wm - o_wm) <= bm
    assert ctx.fields_energy() == (we, wm)  # fixed reduction order
    # zero fields
    ctx.fields_upload(np.zeros(cx.Ne), np.zeros(cx.Nf, np.int64))
    assert ctx.fields_energy() == (0.0, 0.0)

    # source-free steps, Gauss-law solve off
    ctx.fields_upload(e, b)
    w0 = sum(ctx.fields_energy())
    moved = 0.0
    for _ in range(12):
        ctx.pic_step(ctx.step_params(field_mode=qh.FIELDS_SOLVE, gauss=0, tol_edge=1e-12), 1)
        we1, wm1 = ctx.fields_energy()
        w = we1 + wm1
        moved = max(moved, abs(we1 - we))
        assert abs(w - w0) <= 1e-10 * w0
    assert moved > 1e-3 * w0  # energy did pass between the electric and magnetic parts
    e_g, b_g = ctx.fields_download()
    o = oracle_energy(e_g, b_g)
    assert abs(w - (o[0] + o[1])) <= o[2] + o[3]
    # with the Gauss-law solve, from the solenoidal part of e
    _, e_s, _, _ = ctx.fields_decompose(tol=1e-13)
    ctx2 = context()
    ctx2.fields_upload(e_s, b)
    w0 = sum(ctx2.fields_energy())
    for _ in range(12):
        st = ctx2.pic_step(ctx2.step_params(field_mode=qh.FIELDS_SOLVE, tol_edge=1e-12, tol_node=1e-12), 1)[0]
        w = sum(ctx2.fields_energy())
        assert abs(w - w0) <= 1e-10 * w0, st


def test_locate_and_upload_without_tets(jitter4):
    """Point location on the device: every point inside gets a tet holding it (FP64 barycentrics
    of the point in it >= -1e-6; the tet of the brute-force search wherever that one is not
    within 1e-5 of a face); points outside get -1; an upload without tets locates the particles
    and the step that follows keeps continuity."""
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    ctx = gpu_context(mesh, 1e-11)
    ctx.fields_upload(e, b)
    rng = np.random.default_rng(21)
    pts = rng.random((5000, 3))
    t = ctx.locate(pts)
    lam = np.einsum("tij,pj->pti", op.Minv, np.column_stack([np.ones(len(pts)), pts]))
    ref = np.argmax(lam.min(axis=2), axis=1)
    clear = lam.min(axis=2)[np.arange(len(pts)), ref] > 1e-5
    assert (t >= 0).all()
    own = lam[np.arange(len(pts)), t].min(axis=1)
    assert own.min() > -1e-6
    assert (t[clear] == ref[clear]).all()
    outside = pts + np.array([1.5, 0.0, 0.0])
    assert (ctx.locate(outside[:100]) == -1).all()
    x, v, tet = parts["e"]
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    ctx.particles_upload(sid, x, v)
    _, _, tg = ctx.particles_download(sid)
    lam_p = np.einsum("pij,pj->pi", op.Minv[tg], np.column_stack([np.ones(len(x)), x.astype(np.float64)]))
    assert lam_p.min() > -1e-6 and (tg == tet).mean() > 0.99
    st = ctx.pic_step(ctx.step_params(verify=1))[0]
    assert st["continuity_bad"] == 0 and st["lost"] == 0
    bad = x.copy()
    bad[7] = [2.0, 0.5, 0.5]
    with pytest.raises(qh.QhError) as ei:
        ctx.particles_upload(sid, bad, v)
    assert ei.value.code == qh.QH_EINVAL and ctx.particles_count(sid) == 0


class _DeviceBuffers:
    """hipMalloc / hipMemcpy from the HIP runtime the library itself loaded (same process, same
    runtime object), for the device-pointer entry points."""

    def __init__(self):
        import ctypes as C
        self.C = C
        self.hip = C.CDLL("libamdhip64.so.7")
        self.hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        self.hip.hipFree.argtypes = [C.c_void_p]
        self.ptrs = []

    def alloc(self, nbytes):
        p = self.C.c_void_p()
        assert self.hip.hipMalloc(self.C.byref(p), nbytes) == 0
        self.ptrs.append(p.value)
        return p.value

    def put(self, arr):
        arr = np.ascontiguousarray(arr)
        d = self.alloc(arr.nbytes)
        assert self.hip.hipMemcpy(d, arr.ctypes.data, arr.nbytes, 1) == 0   # host to device
        return d

    def get(self, d, like):
        out = np.empty_like(like)
        assert self.hip.hipMemcpy(out.ctypes.data, d, out.nbytes, 2) == 0   # device to host
        return out

    def free(self):
        for p in self.ptrs:
            self.hip.hipFree(p)


def test_device_pointer_transfers(jitter4):
    """Fields and deposits through device pointers (buffers of the library's own HIP runtime;
    stream-ordered copies): the downloads equal the host ones; an upload from device memory
    zeroes PEC wall edges and gives the same step as the host upload of the same fields; a flux
    vector with D b != 0 is refused and leaves the fields as they were."""
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    ctx = gpu_context(mesh, 2e-10)
    ref = gpu_context(mesh, 2e-10)
    dev = _DeviceBuffers()
    try:
        ctx.fields_upload(e, b)
        e_d, b_d = dev.alloc(8 * cx.Ne), dev.alloc(8 * cx.Nf)
        ctx.fields_download_dev(e_d, b_d)
        ctx.fields_download()                      # synchronises the context's stream
        assert np.array_equal(dev.get(e_d, e), e) and np.array_equal(dev.get(b_d, b), b)
        e2 = 2.0 * e
        e2[cx.wall_edge] = 5.0
        ctx.fields_upload_dev(dev.put(e2), b_d)
        expect = 2.0 * e
        expect[cx.wall_edge] = 0.0
        eh, bh = ctx.fields_download()
        assert np.array_equal(eh, expect) and np.array_equal(bh, b)
        b_bad = b.copy()
        b_bad[int(np.flatnonzero(~cx.wall_face)[0])] += 1
        with pytest.raises(qh.QhError) as ei:
            ctx.fields_upload_dev(e_d, dev.put(b_bad))
        assert ei.value.code == qh.QH_EINVAL
        assert np.array_equal(ctx.fields_download()[0], expect)
        # the step after the device upload equals the step after the host upload, bit for bit
        x, v, tet = parts["e"]
        ref.fields_upload(expect, b)
        outs = []
        for c in (ctx, ref):
            sid = c.species_add(-qi.QE / qi.ME, -1)
            c.particles_upload(sid, x, (v * 20).astype(np.float32), tet)
            c.pic_step(c.step_params(field_mode=qh.FIELDS_SOLVE, tol_edge=1e-10, tol_node=1e-10))
            outs.append(c.fields_download() + c.deposits_download())
        for a, r in zip(outs[0], outs[1]):
            assert np.array_equal(a, r)
        g_d, q_d = dev.alloc(8 * cx.Ne), dev.alloc(8 * cx.Nn)
        ctx.deposits_download_dev(g_d, q_d)
        ctx.fields_download()
        assert np.array_equal(dev.get(g_d, outs[0][2]), outs[0][2]) and np.array_equal(dev.get(q_d, outs[0][3]), outs[0][3])
    finally:
        dev.free()


def test_particle_order_does_not_change_the_run(jitter4):
    """Race detector of the integer design: the same particles uploaded in two orders (the tet
    sort keeps them in input order only up to its atomics, so the blocks, mailboxes and walks
    see different arrangements) give bit-identical fields, deposits and particle states (by id)
    over 10 full steps, and so does a second run in the same order."""
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    x, v, tet = parts["e"]
    v = (v * 20).astype(np.float32)
    perm = np.random.default_rng(31).permutation(tet.size)
    runs = []
    for order in (np.arange(tet.size), perm, np.arange(tet.size)):
        ctx = gpu_context(mesh, 2e-10)
        ctx.fields_upload(e, b)
        sid = ctx.species_add(-qi.QE / qi.ME, -1)
        ctx.particles_upload(sid, x[order], v[order], tet[order])
        ctx.pic_step(ctx.step_params(field_mode=qh.FIELDS_SOLVE, sort_every=3, verify=1), 10)
        xs, vs, ts = ctx.particles_download(sid)
        back = np.empty_like(order)
        back[order] = np.arange(order.size)      # id k of this run is particle order[k]
        runs.append(ctx.fields_download() + ctx.deposits_download() + (xs[back], vs[back], ts[back]))
    for r in runs[1:]:
        for a, ref in zip(r, runs[0]):
            assert np.array_equal(a, ref)


def test_checkpoint_resume_is_bit_identical(jitter4):
    """20 steps straight equal 10 steps, a checkpoint, a fresh context loading it, and 10 more,
    bit for bit (fields, deposits, particles by id), in the wave-equation mode (its history of
    e^{n-1} and the previous current is in the checkpoint) with a sort every 4 steps. A
    corrupted blob and one from another species list are refused and change nothing."""
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    x, v, tet = parts["e"]
    v = (v * 20).astype(np.float32)
    prm = qh.Context.step_params(field_mode=qh.FIELDS_WAVE, sort_every=4, verify=1, tol_edge=1e-10, tol_node=1e-10)

    def setup(particles=True):
        c = gpu_context(mesh, 2e-10)
        c.fields_upload(e, b)
        s = c.species_add(-qi.QE / qi.ME, -1)
        if particles:
            c.particles_upload(s, x, v, tet)
            c.charge_background(1)
        return c, s

    def state(c, s):
        return c.fields_download() + c.deposits_download() + c.particles_download(s) + (c.particles_ids(s),)

    a, sa = setup()
    for st in a.pic_step(prm, 20):
        assert st["continuity_bad"] == 0
    ref = state(a, sa)
    h, sh = setup()
    h.pic_step(prm, 10)
    blob = h.state_save()
    assert blob[:8] == b"QHSTATE1"
    r, sr = setup(particles=False)
    r.state_load(blob)
    for st in r.pic_step(prm, 10):
        assert st["continuity_bad"] == 0
    for u, w in zip(state(r, sr), ref):
        assert np.array_equal(u, w)
    bad = bytearray(blob)
    bad[200] ^= 1
    before = r.fields_download()[0]
    with pytest.raises(qh.QhError) as ei:
        r.state_load(bytes(bad))
    assert ei.value.code == qh.QH_EINVAL
    o = gpu_context(mesh, 2e-10)
    o.fields_upload(e, b)
    o.species_add(qi.QE / qi.MI, 1)
    with pytest.raises(qh.QhError) as ei:
        o.state_load(blob)
    assert ei.value.code == qh.QH_EINVAL
    assert np.array_equal(r.fields_download()[0], before)


def test_walk_cap_is_reported_and_keeps_continuity(jitter4):
    """Fault forced from the host: some particles so fast that their path needs more than the
    64-piece walk cap in one step. The step reports QH_ELOST with the count, keeps every
    particle (stopped where the cap hit, inside a tet), and continuity still holds bit for bit
    (the path up to there is deposited and the charge sits at the stopping point)."""
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    x, v, tet = parts["e"]
    v = v.copy()
    v[:50] = np.float32(3e10) * np.array([0.6, 0.48, 0.64], np.float32)   # ~30 m per step in a 1 m box
    ctx = gpu_context(mesh, 1e-9)
    ctx.fields_upload(e, b)
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    ctx.particles_upload(sid, x, v, tet)
    _, Q0 = ctx.deposits_download()
    with pytest.raises(qh.QhError) as ei:
        ctx.pic_step(ctx.step_params(verify=1))
    assert ei.value.code == qh.QH_ELOST
    ctx.particles_upload(sid, x, v, tet)
    _, Q0 = ctx.deposits_download()
    st = ctx.pic_step(ctx.step_params(verify=1), allow=(qh.QH_ELOST,))[0]
    assert st["lost"] == 50 and st["continuity_bad"] == 0
    # the status does not depend on asking for statistics
    ctx.particles_upload(sid, x, v, tet)
    with pytest.raises(qh.QhError) as ei:
        ctx.pic_step(ctx.step_params(verify=1), want_stats=False)
    assert ei.value.code == qh.QH_ELOST
    ctx.particles_upload(sid, x, v, tet)
    _, Q0 = ctx.deposits_download()
    ctx.pic_step(ctx.step_params(verify=1), want_stats=False, allow=(qh.QH_ELOST,))
    g, Q1 = ctx.deposits_download()
    assert np.array_equal(cx.G.T @ g, Q1 - Q0)
    xg, _, tg = ctx.particles_download(sid)
    assert ctx.particles_count(sid) == tet.size
    lam = np.einsum("pij,pj->pi", op.Minv[tg], np.column_stack([np.ones(tet.size), xg.astype(np.float64)]))
    assert lam.min() > -1e-5


def _fnv1a(data: bytes) -> int:
    h = 2166136261
    for byte in data:
        h = ((h ^ byte) * 16777619) & 0xFFFFFFFF
    return h


def _reseal(blob: bytearray) -> bytes:
    """A checkpoint blob edited on purpose, with its FNV-1a checksum recomputed."""
    blob[-4:] = _fnv1a(bytes(blob[:-4])).to_bytes(4, "little")
    return bytes(blob)


def test_verification_failure_is_reported_without_stats(jitter4):
    """Fault forced from the host: a checkpoint whose node charge Q^n is one unit off at one
    interior node (checksum recomputed, so the blob loads). The next step's continuity
    G^T g = Q^{n+1} - Q^n then fails at that node: with verification the call reports
    QH_EVERIFY whether or not statistics are asked for, and the statistics count the node."""
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    x, v, tet = parts["e"]
    c = gpu_context(mesh, cfg["dt"])
    c.fields_upload(e, b)
    sid = c.species_add(-qi.QE / qi.ME, -1)
    c.particles_upload(sid, x, v, tet)
    blob = bytearray(c.state_save())
    node = int(cx.int_nodes[0])
    off = 72 + 8 * (cx.Ne + cx.Nf) + 8 * node
    q = int.from_bytes(blob[off:off + 8], "little", signed=True) + 1
    blob[off:off + 8] = q.to_bytes(8, "little", signed=True)
    bad = _reseal(blob)
    for want_stats in (False, True):
        c.state_load(bad)
        with pytest.raises(qh.QhError) as ei:
            c.pic_step(c.step_params(verify=1), want_stats=want_stats)
        assert ei.value.code == qh.QH_EVERIFY
    c.state_load(bad)
    st = c.pic_step(c.step_params(verify=1), allow=(qh.QH_EVERIFY,))[0]
    assert st["continuity_bad"] == 1 and st["divb_bad"] == 0
    # without verification nothing is checked and the step reports no failure
    c.state_load(bad)
    c.pic_step(c.step_params(verify=0))


def test_state_blob_with_out_of_range_count_is_refused(jitter4):
    """A checkpoint whose species count is 2^31 or 2^62 (checksum recomputed) is refused with
    QH_EINVAL before any size is formed from it, and the context keeps its fields and
    particles."""
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    x, v, tet = parts["e"]
    c = gpu_context(mesh, cfg["dt"])
    c.fields_upload(e, b)
    sid = c.species_add(-qi.QE / qi.ME, -1)
    c.particles_upload(sid, x, v, tet)
    blob = c.state_save()
    before = (c.fields_download()[0], c.particles_download(sid)[0])
    off = 72 + 8 * (cx.Ne + cx.Nf + 2 * cx.Nn) + 16   # species 0: q/m, z, pad, then n
    assert int.from_bytes(blob[off:off + 8], "little") == x.shape[0]
    for n_bad in (1 << 31, 1 << 62, -1):
        bad = bytearray(blob)
        bad[off:off + 8] = n_bad.to_bytes(8, "little", signed=True)
        with pytest.raises(qh.QhError) as ei:
            c.state_load(_reseal(bad))
        assert ei.value.code == qh.QH_EINVAL
    assert np.array_equal(c.fields_download()[0], before[0])
    assert np.array_equal(c.particles_download(sid)[0], before[1])
    c.state_load(blob)


def test_fixed_point_headroom_is_reported(jitter4):
    """Fault forced from the host: 20,000 particles of charge number 64 move together along an
    edge of one tet (barycentrics 0.9/0.05 -> 0.05/0.9). A node's charge in that step is about
    20,000 * 64 * 0.9 * 2^40 > 2^60: the step reports QH_EOVERFLOW while the int64 sums are still
    exact (continuity holds); the same particles with charge number 1 are far below it."""
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    t = int(np.flatnonzero(~np.isin(np.arange(cx.Nt), np.flatnonzero((cx.tet_nbr < 0).any(axis=1))))[0])
    V = cx.xyz[cx.tets[t]]
    p0 = np.array([0.9, 0.05, 0.025, 0.025]) @ V
    p1 = np.array([0.05, 0.9, 0.025, 0.025]) @ V
    n, dt = 20_000, 1e-12
    x = np.tile(p0.astype(np.float32), (n, 1))
    v = np.tile(((p1 - p0) / dt).astype(np.float32), (n, 1))
    tet = np.full(n, t, np.int32)
    for z in (64, 1):
        ctx = gpu_context(mesh, dt)
        ctx.fields_upload(np.zeros(cx.Ne), np.zeros(cx.Nf, np.int64))
        sid = ctx.species_add(-z * qi.QE / qi.ME, -z)
        ctx.particles_upload(sid, x, v, tet)
        if z == 64:
            with pytest.raises(qh.QhError) as ei:
                ctx.pic_step(ctx.step_params(verify=1))
            assert ei.value.code == qh.QH_EOVERFLOW
            ctx.particles_upload(sid, x, v, tet)
        _, Q0 = ctx.deposits_download()
        st = ctx.pic_step(ctx.step_params(verify=1), allow=(qh.QH_EOVERFLOW,))[0]
        assert st["continuity_bad"] == 0
        g, Q1 = ctx.deposits_download()
        assert np.array_equal(cx.G.T @ g, Q1 - Q0)
        assert (np.abs(Q1).max() > 2 ** 60) == (z == 64)


def test_field_solve_residual(jitter4):
    import scipy.sparse.linalg as sla
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    dt = 1e-9
    ctx = gpu_context(mesh, dt)
    ie, inn = cx.int_edges, cx.int_nodes
    rng = np.random.default_rng(9)
    A = (op.Meps + dt * dt / 4 * op.S)[ie][:, ie].tocsc()
    K = op.K[inn][:, inn].tocsc()
    for system, M in ((qh.SYS_EDGE, A), (qh.SYS_NODE, K)):
        rhs = rng.standard_normal(M.shape[0]) * 1e-12
        ref = sla.spsolve(M, rhs)
        # FP64 PCG, and FP32 PCG with FP64 reliable updates (the right-hand side of order 1e-12
        # checks its scaling to a unit residual)
        for solver in (qh.SOLVER_FP64, qh.SOLVER_MIXED):
            x, st = ctx.field_solve(system, rhs, tol=1e-8, solver=solver)
            assert st["res"] <= 1e-8 and st["fallback"] == 0
            assert np.linalg.norm(M @ x - rhs) <= 1.0001e-8 * np.linalg.norm(rhs)
            assert np.linalg.norm(x - ref) <= 1e-5 * np.linalg.norm(ref)


def test_degenerate_particle_sets(jitter4):
    """An empty species, a lone particle, and 513 particles (one full block and one particle)
    holding 120 degenerate starts: on a vertex, a face centroid or an edge midpoint of their tet,
    every fourth one at rest, the rest moving a cell or so. Nothing is lost; the integer deposits
    are the GPU's own pieces re-deposited by the oracle, bit for bit; continuity holds on the
    host; positions and tets agree with the oracle's FP64 push (ties aside)."""
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    dt = 2e-9
    ctx = gpu_context(mesh, dt)
    ctx.fields_upload(e, b)
    x, v, tet = parts["e"]
    rng = np.random.default_rng(11)
    T, k = cx.tets, 40
    tt = rng.integers(cx.Nt, size=k)
    special = np.concatenate([cx.xyz[T[tt, 0]], cx.xyz[T[tt][:, [0, 1, 2]]].mean(axis=1),
                              cx.xyz[T[tt][:, [0, 3]]].mean(axis=1)]).astype(np.float32)
    sets = {"empty": (np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), np.zeros(0, np.int32)),
            "one": (x[:1], (v[:1] * 40).astype(np.float32), tet[:1])}
    xs = np.concatenate([special, x[1:1 + 513 - 3 * k]])
    vs = (v[1:514] * 40).astype(np.float32)
    vs[:3 * k:4] = 0.0
    ts = np.concatenate([np.tile(tt, 3), tet[1:1 + 513 - 3 * k]]).astype(np.int32)
    sets["many"] = (xs, vs, ts)
    sids = {}
    for name, (xx, vv, tq) in sets.items():
        sids[name] = ctx.species_add(-qi.QE / qi.ME, -1)
        ctx.particles_upload(sids[name], xx, vv, tq)
    _, Q0 = ctx.deposits_download()
    ctx.capture_segments(64 * 600)
    st = ctx.pic_step(ctx.step_params(verify=1))[0]
    assert st["lost"] == 0 and st["continuity_bad"] == 0
    g, Q1 = ctx.deposits_download()
    assert np.array_equal(cx.G.T @ g, Q1 - Q0)
    nseg, seg = ctx.segments_download()
    assert nseg == seg["tet"].size and np.unique(seg["species"]).size == 2
    g_re, _ = po.deposit_list(seg["tet"], seg["lam0"], seg["lam1"], -np.ones(nseg), np.zeros(0),
                              np.zeros((0, 4)), np.zeros(0))
    assert np.array_equal(g_re, g)
    order = np.lexsort((seg["seq"], seg["pid"], seg["species"]))
    key = seg["species"][order].astype(np.int64) << 32 | seg["pid"][order]
    last = np.r_[key[1:] != key[:-1], True]
    assert last.sum() == 514
    _, Q_re = po.deposit_list(np.zeros(0), np.zeros((0, 4)), np.zeros((0, 4)), np.zeros(0),
                              seg["tet"][order][last], seg["lam1"][order][last], -np.ones(last.sum()))
    assert np.array_equal(Q_re, Q1)
    for name, (xx, vv, tq) in sets.items():
        xg, vg, tg = ctx.particles_download(sids[name])
        assert xg.shape[0] == tq.size
        if tq.size == 0:
            continue
        orc = po.push(e, b * U_B, xx, vv, tq, -qi.QE / qi.ME, dt, -1)
        same = tg == orc["tet"]
        assert same.mean() > 0.95
        assert np.abs(xg - orc["x"]).max(axis=1)[same].max() < 1e-5


def test_gauss_correction_holds_the_law(jitter4):
    """Sec. I, Sec. V: with a loose edge solve (relative residual 1e-4) the error of the discrete
    Gauss law is orders of magnitude above the node solve's tolerance when the correction is
    skipped, and stays within that tolerance (1e-8) when it runs. The error the library reports equals the oracle's
    evaluation of the law on the library's own e and Q. The start satisfies the law exactly
    (E = 0, neutralising background)."""
    import paper_2103_06737_amd as qh
    from oracle.field import FieldOracle
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    dt = cfg["dt"]
    u_q = qi.QE * 2.0 ** -40
    fo = FieldOracle(cx, op, dt)
    res = {}
    for gauss in (1, 0):
        ctx = gpu_context(mesh, dt)
        ctx.fields_upload(np.zeros_like(e), b)
        sid = ctx.species_add(-qi.QE / qi.ME, -1)
        x, v, tet = parts["e"]
        ctx.particles_upload(sid, x, v, tet)
        ctx.charge_background(1)
        _, Q_bg = ctx.deposits_download()
        prm = ctx.step_params(field_mode=qh.FIELDS_SOLVE, gauss=gauss, tol_edge=1e-4, tol_node=1e-8, verify=1)
        st = ctx.pic_step(prm, 30)
        assert all(s["continuity_bad"] == 0 and s["divb_bad"] == 0 for s in st)
        res[gauss] = np.array([s["gauss_res"] for s in st])
        e1, _ = ctx.fields_download()
        _, Q1 = ctx.deposits_download()
        rho = u_q * (Q_bg - Q1).astype(np.float64)[cx.int_nodes]
        assert abs(fo.gauss_error(e1, rho) - res[gauss][-1]) <= 1e-4 * res[gauss][-1] + 1e-14
    assert res[1].max() <= 1.01e-8
    assert res[0][2:].min() > 1e3 * res[1].max()


def test_wave_gauss_error_grows_without_correction(jitter4):
    """The Gauss-law figure of Sec. VI on the device: with a loose edge solve (1e-4) and no
    correction, the Gauss-law error of the trapezoidal update levels off while that of the
    wave-equation update keeps growing (the t grad Phi null space); with the correction the
    wave-equation update holds the law to the node solve's tolerance."""
    import paper_2103_06737_amd as qh
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    x, v, tet = parts["e"]
    res = {}
    for mode, gauss in ((qh.FIELDS_SOLVE, 0), (qh.FIELDS_WAVE, 0), (qh.FIELDS_WAVE, 1)):
        ctx = gpu_context(mesh, cfg["dt"])
        ctx.fields_upload(np.zeros_like(e), b)
        sid = ctx.species_add(-qi.QE / qi.ME, -1)
        ctx.particles_upload(sid, x, v, tet)
        ctx.charge_background(1)
        st = ctx.pic_step(ctx.step_params(field_mode=mode, gauss=gauss, tol_edge=1e-4, tol_node=1e-8), 40)
        res[mode, gauss] = np.array([s["gauss_res"] for s in st])
    t, w = res[qh.FIELDS_SOLVE, 0], res[qh.FIELDS_WAVE, 0]
    assert t[-1] < 1.2 * t[2]
    assert w[-1] > 3 * w[2] and w[-1] > 3 * t[-1]
    assert res[qh.FIELDS_WAVE, 1].max() <= 1.01e-8


def test_scattered_numbering_reads_wide_column_tiles():
    """Nodes numbered at random on a 24^3 box: the columns of a product tile then scatter over
    the whole range of ~97 K interior edges, more than four 2^14-column windows hold, so the
    products of the edge matrix and of the learned factor read 32-bit columns. Both edge solves
    still reach the relative residual 1e-8 against the oracle's FP64 matrix."""
    import paper_2103_06737_amd as qh
    from oracle.complex_ import Complex
    from oracle.whitney import Operators
    mesh = qi.make_mesh(dict(n=24, jitter=0.0, z_ratio=1.0))
    perm = np.random.default_rng(3).permutation(mesh.xyz.shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    xyz, tets = mesh.xyz[perm], inv[mesh.tets].astype(np.int32)
    dt = 1e-10
    ctx = qh.Context(0)
    ctx.mesh_upload(xyz, tets)
    ctx.set_physics(qi.EPS0, qi.MU0, dt, qi.QE * 2.0 ** -40, 2.0 ** -56)
    mi = ctx.mesh_info()
    assert mi.n_int_edges > 65536 and mi.nnz_edge_c16 < mi.nnz_edge // 2
    cx = Complex(xyz, tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    ie = cx.int_edges
    A = (op.Meps + dt * dt / 4 * op.S)[ie][:, ie].tocsr()
    rhs = np.random.default_rng(4).standard_normal(ie.size) * 1e-12
    x, st = ctx.field_solve(qh.SYS_EDGE, rhs, tol=1e-8)
    assert np.linalg.norm(A @ x - rhs) <= 1.0001e-8 * np.linalg.norm(rhs)
    ctx.precond_train(steps=20, lr=3e-3, seed=1, validate_every=0)
    mi = ctx.mesh_info()
    assert 0 < mi.nnz_factor and mi.nnz_factor_c16 < 2 * mi.nnz_factor  # G and G^T together
    xl, stl = ctx.field_solve(qh.SYS_EDGE, rhs, tol=1e-8, precond=qh.PC_LEARNED)
    assert stl["fallback"] == 0 and stl["iters"] < st["iters"]
    assert np.linalg.norm(A @ xl - rhs) <= 1.0001e-8 * np.linalg.norm(rhs)
    # the FP32 inner iterations of the mixed solve through the same 32-bit column tiles
    for pc in (qh.PC_JACOBI, qh.PC_LEARNED):
        xm, stm = ctx.field_solve(qh.SYS_EDGE, rhs, tol=1e-8, precond=pc, solver=qh.SOLVER_MIXED)
        assert stm["fallback"] == 0
        assert np.linalg.norm(A @ xm - rhs) <= 1.0001e-8 * np.linalg.norm(rhs)


def test_sort_keeps_particles_and_invariants(jitter4):
    cfg, mesh, cx, op, po, e, b, parts = jitter4
    ctx = gpu_context(mesh, 2e-9)
    ctx.fields_upload(e, b)
    sid = ctx.species_add(-qi.QE / qi.ME, -1)
    x, v, tet = parts["e"]
    ctx.particles_upload(sid, x, (v * 40).astype(np.float32), tet)
    a = ctx.pic_step(ctx.step_params(sort_every=1, verify=1), 3)
    assert all(s["continuity_bad"] == 0 for s in a)
    xs, vs, ts = ctx.particles_download(sid)
    ctx2 = gpu_context(mesh, 2e-9)
    ctx2.fields_upload(e, b)
    sid2 = ctx2.species_add(-qi.QE / qi.ME, -1)
    ctx2.particles_upload(sid2, x, (v * 40).astype(np.float32), tet)
    ctx2.pic_step(ctx2.step_params(sort_every=0), 3)
    xu, vu, tu = ctx2.particles_download(sid2)
    # the per-particle result does not depend on the storage order
    assert np.array_equal(xs, xu) and np.array_equal(vs, vu) and np.array_equal(ts, tu)
