#!/usr/bin/env python3
"""Benchmark: one full PIC cycle per step of the 64^3 uniform-plasma workload on one MI355X.

Workload: unit cube, 64^3 boxes x 6 Kuhn tets (1,572,864 tets, 1,872,064 edges), 16,000,000
electrons (uniform, Maxwellian v_th = 1e6 m/s, n = 1e16 m^-3, neutralising background),
uniform B_z = 0.1 T, dt = 1.2e-10 s (~10x the explicit limit), counting sort by tet every 20
steps, full cycle: gather + Boris + tet walk + int64 deposit, then the implicit field update
(edge CG to 1e-8, Gauss-law CG to 1e-8, integer Faraday). Synthetic seeded inputs.

Prints one JSON line. value = particle-steps/s of the whole cycle (N_p * K / wall time of K
steps, inputs resident on the GPU). Extra keys give the particle phase and the field solve
separately, per-kernel device times (HIP events), the roofline of the dominant kernel and
the FP64 oracle timed on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import qh_inputs as qi  # noqa: E402

HBM_PEAK_GBS = 8000.0
WORKLOADS = {"plasma64": "64^3 Kuhn cube, 16M-electron uniform plasma, full implicit cycle",
             "beam32": "32^3 Kuhn cube, 1M-electron beam in frozen random fields",
             "graded96": "96^3 Kuhn cube graded toward z=0 (ratio 1.05), 32M electrons + 32M ions, full implicit cycle"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup(wl: str, n_particles: int | None, boundary: int = 0, seed: int = 0, **override):
    import paper_2103_06737_amd as qh
    cfg = dict(qi.CONFIGS[wl], **override)
    mesh = qi.make_mesh(cfg)
    n_e = cfg["n_e"] if n_particles is None else n_particles
    weight = cfg["weight"] * cfg["n_e"] / n_e
    t0 = time.perf_counter()
    ctx = qh.Context(0)
    ctx.set_boundary(boundary)
    ctx.mesh_upload(mesh.xyz, mesh.tets)
    u_b = 2.0 ** -56
    ctx.set_physics(qi.EPS0, qi.MU0, cfg["dt"], qi.QE * weight * 2.0 ** -40, u_b)
    mi = ctx.mesh_info()
    ctx.fields_init_synthetic(qi.white(mi.n_edges, 0, 3), qi.white(mi.n_edges, 0, 5), cfg["sigma_e"], cfg["bz"],
                              cfg["sigma_b"])
    log(f"[bench] mesh + assembly {time.perf_counter() - t0:.1f}s  tets={mi.n_tets} edges={mi.n_edges} "
        f"nnz_edge={mi.nnz_edge}")
    t0 = time.perf_counter()
    parts = qi.make_particles(mesh, cfg, seed=seed, n_e=n_e)
    sids = []
    for name, (x, v, tet) in parts.items():
        qm, z = (-qi.QE / qi.ME, -1) if name == "e" else (qi.QE / qi.MI, 1)
        sid = ctx.species_add(qm, z)
        ctx.particles_upload(sid, x, v, tet)
        sids.append(sid)
    if cfg["mode"] == "solve":
        ctx.charge_background(1)
    log(f"[bench] particles {time.perf_counter() - t0:.1f}s  n={sum(p[2].size for p in parts.values())}")
    return ctx, cfg, mesh, parts, mi


def phase_bytes(mi, n_particles: int, crossings: float, n_occ: int) -> int:
    """Algorithmic bytes of one particle phase (gather, push, walk, deposit): the particle state
    read and written once (x, v as FP32 and the tet as int32: 56 B), per occupied tet and per
    further tet a crossing enters the FP32 geometry (64 B), the E/B record (40 B), node and edge
    ids (40 B) and neighbours (16 B), and the int64 edge and node accumulators written once."""
    return 56 * n_particles + 160 * n_occ + 160 * crossings + 16 * (mi.n_edges + mi.n_nodes)


def algorithmic_bytes(kernel: str, mi, n_particles: int, crossings: float, learned: bool = False,
                      mixed: bool = False, n_species: int = 1):
    """Bytes one launch must move at least (each datum read or written once). mixed: the inner
    iterations of the mixed-precision edge solve (FP32 matrix values and vectors)."""
    v = 4 if mixed else 8   # bytes per vector entry (and per value of A) in the edge iterations
    if kernel in ("cg_spmv",):
        # A: value + column (2 bytes in tiles read with 16-bit offsets, else 4); rowptr;
        # z, p_old, q_old in; p_new, q out
        n, nnz, c16 = mi.n_int_edges, mi.nnz_edge, mi.nnz_edge_c16
        return v * nnz + 2 * c16 + 4 * (nnz - c16) + 4 * (n + 1) + 5 * v * n
    if kernel in ("node_spmv",):
        n, nnz = mi.n_int_nodes, mi.nnz_node
        return 12 * nnz + 4 * (n + 1) + 32 * n
    if kernel == "node_update":
        return 64 * mi.n_int_nodes
    if kernel == "cg_update":
        n = mi.n_int_edges
        if learned:
            return 6 * v * n                             # x, r rw; p, q in (z comes from the factor)
        return 8 * v * n                                 # x, r rw; p, q, dinv in; z out
    if kernel == "particle_step":
        # one launch per species: particle state in+out (28 B each way), per tet: geometry 48 +
        # field 48 + vertex ids 16 + edge ids 24, per crossing: neighbour ids 16 + the next tet's
        # records 136, accumulators read-modify-write once (16 B per edge and node); n_particles
        # and crossings are the step's totals, and the result is the average launch's share
        per_step = (56 * n_particles + n_species * (136 * mi.n_tets + 16 * (mi.n_edges + mi.n_nodes))
                    + 152 * crossings)
        return per_step / n_species
    if kernel == "precond":
        # z = G^T (G r): two CSR passes over the lower factor and its transpose (BF16 value,
        # column of 2 or 4 bytes as in cg_spmv); per row: r in, y out, y in, z out, r in (dot),
        # row pointers
        n, nnz_l, c16 = mi.n_int_edges, mi.nnz_factor, mi.nnz_factor_c16
        return 4 * nnz_l + 2 * c16 + 4 * (2 * nnz_l - c16) + 5 * v * n + 8 * (n + 1)
    if kernel == "field_prep":
        return (48 + 24 + 16 + 48) * mi.n_tets + 8 * mi.n_edges + 8 * mi.n_faces
    return None


# HIP kernels behind each timed entry (one entry may launch several kernels)
HIP_KERNELS = {"particle_step": ["k_particle_step<false>", "k_mail_apply", "k_gather<0, 2>", "k_gather<6, 8>"],
               "edge_rhs": ["k_edge_rhs_e", "k_edge_rhs_b"], "field_prep": ["k_field_prep"]}


def hip_kernels(entry: str, mixed: bool = False, learned: bool = False):
    """HIP kernels behind a timed entry; the edge iterations' kernels are instantiated on FP64
    vectors, or FP32 in the mixed-precision solve, and the update computes z = D^-1 r only with
    Jacobi."""
    t = "float" if mixed else "double"
    if entry == "cg_spmv":
        return [f"k_cg_spmv<{t}, {t}>"]
    if entry == "cg_update":
        return [f"k_cg_update<{'false' if learned else 'true'}, {t}>"]
    if entry == "precond":
        return [f"k_prec_g<false, {t}>", f"k_prec_g<true, {t}>"]
    return HIP_KERNELS.get(entry, [])


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_plasma_64cube_16M.md")
# headers every kernel file includes: part of the source a traffic figure was taken from
SHARED_SOURCES = ["paper_2103_06737_amd/csrc/qh_spmv.h", "paper_2103_06737_amd/csrc/qh_internal.h"]


def measured_traffic(entry: str, workload: str, kernels):
    """HBM bytes per launch from the profiler's byte counters (scaled by the copy calibration),
    as recorded in the traffic summary; None when the summary is absent, covers another
    workload, or any kernel's source (its file and the shared headers) has changed since the
    counters were taken."""
    import hashlib
    if workload != "plasma64" or not kernels or not os.path.exists(TRAFFIC_FILE):
        return None
    rows = {}
    for line in open(TRAFFIC_FILE):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 6 and cells[0].startswith("`k_"):
            src = cells[5].split()
            rows[cells[0].strip("`")] = (float(cells[4]) * 1e6, src)
    total = 0.0
    for k in kernels:
        if k not in rows or len(rows[k][1]) != 2:
            return None
        path, digest = rows[k][1]
        data = b""
        for p in [path] + SHARED_SOURCES:
            with open(os.path.join(ROOT, p), "rb") as fh:
                data += fh.read()
        if hashlib.sha256(data).hexdigest()[:16] != digest:
            return None
        total += rows[k][0]
    return int(total)


def gauss_study(workload: str, particles, steps: int, tols):
    """Gauss-law error per step of the full cycle with and without the Gauss-law correction, at
    loose edge-solve tolerances, for the trapezoidal (E-B) update and the wave-equation update
    (Sec. I, Sec. V, the Gauss-law figure of Sec. VI: without the correction the solver's error in
    the irrotational part of e is never removed; it levels off for the E-B update and grows in
    time for the wave equation; with it the discrete law holds to the node solve's tolerance
    every step). Each run starts from the same seeded state."""
    import paper_2103_06737_amd as qh
    runs = []
    for tol, mode, gauss in [(t, m, g) for t in tols for m in (qh.FIELDS_SOLVE, qh.FIELDS_WAVE) for g in (1, 0)]:
        ctx, cfg, mesh, parts, mi = setup(workload, particles)
        prm = qh.Context.step_params(field_mode=mode, sort_every=cfg.get("sort_every", 0), gauss=gauss,
                                     tol_edge=tol, tol_node=1e-8, max_it_edge=2000, max_it_node=5000,
                                     check_every=16)
        st = ctx.pic_step(prm, steps)
        runs.append({"update": "wave" if mode == qh.FIELDS_WAVE else "trapezoidal",
                     "tol_edge": tol, "gauss_correction": bool(gauss),
                     "gauss_res": [s["gauss_res"] for s in st],
                     "edge_iters": [s["edge_iters"] for s in st], "node_iters": [s["node_iters"] for s in st]})
        log(f"[study] {runs[-1]['update']} tol_edge {tol:g} correction {bool(gauss)}: "
            f"gauss_res step 1 {st[0]['gauss_res']:.3e}, step {steps} {st[-1]['gauss_res']:.3e}")
        ctx.close()
    print(json.dumps({"study": "gauss_law_error_per_step", "workload": f"{workload}: {WORKLOADS[workload]}",
                      "steps": steps, "tol_node": 1e-8, "runs": runs}))


def boundary_counts(tets: np.ndarray, n_nodes: int):
    """Wall faces (faces of one tet only), their edges and nodes, for the byte count of the
    plane-wave kernels."""
    face_of = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))
    f = np.sort(np.concatenate([tets[:, list(k)] for k in face_of]).astype(np.int64), axis=1)
    key = (f[:, 0] * n_nodes + f[:, 1]) * n_nodes + f[:, 2]
    u, cnt = np.unique(key, return_counts=True)
    wall = u[cnt == 1]
    a, r = np.divmod(wall, n_nodes * n_nodes)
    b, c = np.divmod(r, n_nodes)
    ek = np.unique(np.concatenate([a * n_nodes + b, a * n_nodes + c, b * n_nodes + c]))
    return {"faces": int(wall.size), "edges": int(ek.size), "nodes": int(np.unique(np.concatenate([a, b, c])).size),
            "points": int(18 * wall.size)}


def plane_wave_run(workload: str, particles, steps: int, f0=300e6, bw=150e6, e_peak=1e3):
    """The full cycle with natural walls (all edges and nodes unknowns; the Gauss-law system is
    singular and solved on the consistent right-hand side) driven by a plane-wave pulse through
    the walls (Sec. II.C, Sec. VI.A.2): the boundary term of Ampere's law in the edge right-hand
    side every step and its normal flux in the Gauss-law target. Times the cycle and the two
    boundary kernels, and reports the Gauss-law residual and the solver iterations. The plasma
    starts unmagnetised: natural walls carry no surface current, so the workload's static
    uniform B_z would not be an equilibrium (its wall edges see the whole jump of H)."""
    import paper_2103_06737_amd as qh
    ctx, cfg, mesh, parts, mi = setup(workload, particles, boundary=qh.BC_NEUMANN, bz=0.0)
    n_p = sum(p[2].size for p in parts.values())
    t0 = 4.0 / (2 * np.pi * bw)
    E0 = e_peak / (2 * np.pi * f0)   # E_inc = E0 s'(t - x/c); s' peaks near 2 pi f0
    ctx.set_plane_wave(E0, f0, bw, t0)
    tst = ctx.precond_train(steps=150, lr=3e-3, seed=1, validate_every=0)
    prm = qh.Context.step_params(field_mode=qh.FIELDS_SOLVE, precond=qh.PC_LEARNED,
                                 sort_every=cfg.get("sort_every", 0), tol_edge=1e-8, tol_node=1e-8,
                                 max_it_edge=2000, max_it_node=5000, check_every=16)
    ctx.timing(True)
    w0 = time.perf_counter()
    st = ctx.pic_step(prm, steps)
    wall = time.perf_counter() - w0
    kt = ctx.timing_read()
    ctx.timing(False)
    bc = boundary_counts(mesh.tets, mi.n_nodes)
    ms_b, n_b = kt["boundary"]
    # per wall edge: row pointer, edge id, right-hand side in and out, h sum out; per rule point:
    # coefficient and index of its x (the table of s' per distinct x stays in L2); per wall node:
    # list pointer, node id, flux in and out; per list entry: edge index and its h sum
    by = 32 * bc["edges"] + 12 * bc["points"] + 24 * bc["nodes"] + 12 * 2 * bc["edges"]
    us = 1e3 * ms_b / max(n_b, 1)
    kern = {k: {"ms_total": round(ms, 4), "launches": c, "us_per_launch": round(1e3 * ms / c, 3)}
            for k, (ms, c) in kt.items() if c}
    out = {"study": "plane_wave_natural_boundary", "workload": f"{workload}: {WORKLOADS[workload]}",
           "particles": n_p, "steps": steps, "dt": cfg["dt"], "bz": cfg["bz"],
           "wave": {"E0": E0, "peak_field_approx_V_per_m": e_peak, "f0": f0, "bandwidth": bw, "t0": t0, "polarisation": "-z", "direction": "+x"},
           "boundary": bc, "ms_per_step": round(1e3 * wall / steps, 4),
           "note": "wall time with the per-kernel HIP event pairs recorded (about 4 % over an untimed run)",
           "boundary_kernels": {"us_per_launch": round(us, 3), "algorithmic_bytes_per_launch": by,
                                "achieved_GBs": round(by / (us * 1e-6) / 1e9, 1) if us > 0 else None,
                                "peak_GBs": HBM_PEAK_GBS},
           "edge_iters": [s["edge_iters"] for s in st], "node_iters": [s["node_iters"] for s in st],
           "edge_res_max": max(s["edge_res"] for s in st), "gauss_res_max": max(s["gauss_res"] for s in st),
           "lost": sum(s["lost"] for s in st), "kernels": kern,
           "train": tst}
    log(f"[plane-wave] {out['ms_per_step']} ms/step, boundary {us:.2f} us/launch, gauss_res max "
        f"{out['gauss_res_max']:.2e}, node iters {out['node_iters'][:3]}..{out['node_iters'][-3:]}")
    ctx.close()
    print(json.dumps(out))


def beam_run(steps: int, tol_edge: float = 1e-6):
    """The beam of Sec. VI.B: electrons injected through the z = 0 face of a PEC cylinder
    (radius 20 mm, length 100 mm; 10 macro-particles of 52012.58 electrons per step at the full
    0.25 A, v_p = 5e7 m/s inside r_b = 8 mm, current turned on linearly over 2 ns; absorbing
    walls). Four runs: the trapezoidal (E-B) and wave-equation updates, each with and without
    the Gauss-law correction, at a loose edge tolerance. Per run: time per step (injection,
    cycle and the per-step sort; the stats of every step are read), the radial E halfway down
    the tube at r = 16 mm (the paper's observable, mean of four probes), and the Gauss-law
    error, sampled in time."""
    import paper_2103_06737_amd as qh
    c = qi.BEAM_CYL
    mesh = qi.CylinderMesh(c["R"], c["L"], c["nr"], c["nz"])
    dt = c["dt"]
    counts = qi.beam_injection_counts(steps, dt, c["per_step"], c["t_on"])
    inj = [qi.beam_injection(mesh, int(n), c["r_b"], c["v_p"], seed=0, step=k) if n else None
           for k, n in enumerate(counts)]
    rp = 0.016
    probe = np.array([[rp, 0, 0.5 * c["L"]], [0, rp, 0.5 * c["L"]], [-rp, 0, 0.5 * c["L"]], [0, -rp, 0.5 * c["L"]]])
    ptet = mesh.locate(probe).astype(np.int32)
    rhat = probe[:, :2] / rp
    every = max(1, steps // 40)
    runs = []
    for mode, gauss in ((qh.FIELDS_SOLVE, 1), (qh.FIELDS_WAVE, 1), (qh.FIELDS_SOLVE, 0), (qh.FIELDS_WAVE, 0)):
        ctx = qh.Context(0)
        ctx.set_walls(qh.WALLS_ABSORB)
        ctx.mesh_upload(mesh.xyz, mesh.tets)
        ctx.set_physics(qi.EPS0, qi.MU0, dt, qi.QE * c["weight"] * 2.0 ** -40, 2.0 ** -56)
        mi = ctx.mesh_info()
        ctx.fields_upload(np.zeros(mi.n_edges), np.zeros(mi.n_faces, np.int64))
        sid = ctx.species_add(-qi.QE / qi.ME, -1)
        prm = qh.Context.step_params(field_mode=mode, gauss=gauss, tol_edge=tol_edge, tol_node=1e-8,
                                     max_it_edge=2000, max_it_node=5000, check_every=8)
        t_step, series, absorbed, it_e, it_n = 0.0, [], 0, 0, 0
        for k in range(steps):
            w0 = time.perf_counter()
            if inj[k] is not None:
                ctx.particles_inject(sid, *inj[k])
            st = ctx.pic_step(prm)[0]
            t_step += time.perf_counter() - w0
            absorbed += st["wall_hits"]
            it_e += st["edge_iters"]
            it_n += st["node_iters"]
            if (k + 1) % every == 0:
                E, _ = ctx.probe_fields(probe, ptet)
                er = float(np.mean(np.sum(E[:, :2] * rhat, axis=1)))
                series.append([round((k + 1) * dt * 1e9, 4), er, st["gauss_res"], ctx.particles_count(sid)])
        runs.append({"update": "wave" if mode == qh.FIELDS_WAVE else "trapezoidal", "gauss_correction": bool(gauss),
                     "ms_per_step": round(1e3 * t_step / steps, 4), "injected": int(counts.sum()),
                     "absorbed": int(absorbed), "in_flight": ctx.particles_count(sid),
                     "edge_iters_mean": round(it_e / steps, 2), "node_iters_mean": round(it_n / steps, 2),
                     "samples_t_ns_Er_gaussres_count": series})
        log(f"[beam] {runs[-1]['update']} correction {bool(gauss)}: {runs[-1]['ms_per_step']} ms/step, "
            f"in flight {runs[-1]['in_flight']}, absorbed {absorbed}, E_r end {series[-1][1]:.4g} V/m, "
            f"gauss_res end {series[-1][2]:.3e}")
        ctx.close()
    print(json.dumps({"study": "beam_injection_cylinder", "workload": "PEC cylinder r 20 mm x 100 mm "
                      f"({mesh.tets.shape[0]} tets), beam of the Sec. VI.B table", "steps": steps, "dt": dt,
                      "tol_edge": tol_edge, "tol_node": 1e-8, "probe": "E_r at z = 50 mm, r = 16 mm",
                      "runs": runs}))


def cpu_baseline(wl: str, cfg, mesh, parts, sample_particles: int, seconds_cap: float = 25.0):
    """The FP64 oracle as it stands, on the host cores: one particle push over a sample of the
    particles plus one oracle field update on the full mesh; whole-step rate extrapolated to
    the full particle count."""
    from oracle.complex_ import Complex
    from oracle.field import FieldOracle
    from oracle.particles import ParticleOracle
    from oracle.whitney import Operators
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    cores = min(cores, 16)
    cx = Complex(mesh.xyz, mesh.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    po = ParticleOracle(cx, op.Minv)
    from oracle.field import init_fields
    u_b = 2.0 ** -56
    e, b = init_fields(cx, qi.white(cx.Ne, 0, 3), qi.white(cx.Ne, 0, 5), cfg["sigma_e"], cfg["bz"], cfg["sigma_b"], u_b)
    x, v, tet = parts["e"]
    n_s = min(sample_particles, tet.size)
    t0 = time.perf_counter()
    out = po.push(e, b * u_b, x[:n_s], v[:n_s], tet[:n_s], -qi.QE / qi.ME, cfg["dt"], -1, nthreads=cores)
    t_push = time.perf_counter() - t0
    n_total = sum(p[2].size for p in parts.values())
    t_field = 0.0
    if cfg["mode"] == "solve":
        fo = FieldOracle(cx, op, cfg["dt"])
        weight = cfg["weight"]
        u_q = qi.QE * weight * 2.0 ** -40
        Q = np.zeros(cx.Nn, np.int64)
        t0 = time.perf_counter()
        fo.step(e, b, u_b, out["g"], u_q, out["Q"], out["Q"], tol=1e-8, tol_n=1e-8)
        t_field = time.perf_counter() - t0
    t_step = t_push * n_total / n_s + t_field
    # the same on one thread: the push over a sample as many times smaller as there were threads
    # (about the same seconds), the field update as above (its sparse products run on one thread)
    n_1 = max(min(n_s, 10_000), n_s // cores)
    t0 = time.perf_counter()
    po.push(e, b * u_b, x[:n_1], v[:n_1], tet[:n_1], -qi.QE / qi.ME, cfg["dt"], -1, nthreads=1)
    t_push1 = time.perf_counter() - t0
    t_step1 = t_push1 * n_total / n_1 + t_field
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": n_total / t_step, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "push_s": round(t_push, 3), "field_s": round(t_field, 3),
            "sample": f"one step of {n_s} of {n_total} particles (FP64 C oracle, {cores} threads, "
                      f"{t_push:.2f}s) + one FP64 field update on the full mesh (numpy/scipy sparse "
                      f"products and PCG, one thread, {t_field:.2f}s); rate = N_p / (push time scaled "
                      f"to N_p + field time)",
            "single_thread": {"value": n_total / t_step1, "unit": "particle-steps/s", "cores": 1,
                              "push_s": round(t_push1, 3), "push_particles": n_1, "field_s": round(t_field, 3),
                              "push_only_particle_steps_per_s": round(n_1 / t_push1, 1)},
            "push_only_particle_steps_per_s": round(n_s / t_push, 1)}


def frozen_particle_phase(workload: str, warmup: int, steps: int):
    """The particle phase alone in frozen fields (the 32^3 beam workload: 1M electrons, its 200
    steps), timed per step with the library's HIP events (field prep, push, walk, deposit and the
    particles' moves between blocks), with its roofline on the phase's algorithmic bytes. Its
    particle state (28 MB) and mesh records fit the 256 MB last-level cache: the bytes need not
    all come from HBM."""
    import paper_2103_06737_amd as qh
    ctx, cfg, mesh, parts, mi = setup(workload, None)
    n_p = sum(p[2].size for p in parts.values())
    n_occ = int(np.unique(np.concatenate([p[2] for p in parts.values()])).size)
    prm = qh.Context.step_params(field_mode=qh.FIELDS_FROZEN, sort_every=cfg.get("sort_every", 0))
    ctx.pic_step(prm, warmup, want_stats=False)
    st = ctx.pic_step(prm, steps, want_stats=True)
    ms = float(np.mean([s["ms_particles"] for s in st]))
    cross = float(np.mean([s["crossings"] for s in st]))
    by = phase_bytes(mi, n_p, cross, n_occ)
    ach = by / (ms * 1e-3) / 1e9
    ctx.close()
    return {"workload": f"{workload}: {WORKLOADS[workload]}", "particles": n_p, "steps": steps,
            "ms_per_step": round(ms, 4), "particle_steps_per_s": round(n_p / (ms * 1e-3), 1),
            "crossings_per_step": cross, "occupied_tets": n_occ,
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_step": int(by),
                         "note": "state and records fit the 256 MB last-level cache"}}


def copy_calibration(mib: int, reps: int = 5):
    """A plain elementwise copy of known size (reads and writes mib MiB once per launch): the
    profiler's FETCH_SIZE / WRITE_SIZE for this kernel, divided by the known bytes, gives the
    factor that turns those counters into HBM bytes."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)  # load the kernel before timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)   # one read and one write of every element
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_calibration": {"bytes_read": 4 * n, "bytes_written": 4 * n, "launches": reps + 1,
                                           "GB_per_s": round(8 * n / dt / 1e9, 1)}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="plasma64", choices=sorted(WORKLOADS))
    ap.add_argument("--particles", type=int, default=None, help="override the particle count")
    ap.add_argument("--profile-steps", type=int, default=None,
                    help="steps timed per kernel with stats (default: one whole re-sort cycle)")
    ap.add_argument("--no-frozen", action="store_true", help="skip the frozen-field beam32 particle phase")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000)
    ap.add_argument("--precond", default="learned", choices=["learned", "jacobi"])
    ap.add_argument("--solver", default="mixed", choices=["mixed", "fp64"],
                    help="edge solve of the headline run: FP64 PCG, or FP32 PCG with FP64 reliable updates; "
                         "both stop on the FP64 residual 1e-8 and both are timed")
    ap.add_argument("--train-steps", type=int, default=150)
    ap.add_argument("--pairs", type=int, default=2000,
                    help="(rhs, solution) pairs of the plain solver recorded for training (particle seed 1; "
                         "0: train on probes only)")
    ap.add_argument("--pair-weight", type=float, default=0.5)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (read + write) a few times, to "
                         "scale the HBM byte counters of the profiler; prints its own JSON line")
    ap.add_argument("--gauss-study", type=int, default=0, metavar="STEPS",
                    help="Gauss-law error per step of the trapezoidal and wave-equation updates with "
                         "and without the correction at loose edge tolerances (1e-4, 1e-6); prints its "
                         "own JSON line")
    ap.add_argument("--plane-wave", type=int, default=0, metavar="STEPS",
                    help="the full cycle with natural walls and a plane-wave pulse entering through them; "
                         "prints its own JSON line")
    ap.add_argument("--beam", type=int, default=0, metavar="STEPS",
                    help="the beam injected into the cylindrical cavity (trapezoidal and wave updates, "
                         "with and without the Gauss-law correction); prints its own JSON line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gauss_study:
        gauss_study(args.workload, args.particles, args.gauss_study, (1e-4, 1e-6))
        return
    if args.plane_wave:
        plane_wave_run(args.workload, args.particles, args.plane_wave)
        return
    if args.beam:
        beam_run(args.beam)
        return
    import paper_2103_06737_amd as qh
    frozen = None
    if not args.no_frozen and args.workload == "plasma64":
        frozen = frozen_particle_phase("beam32", 10, qi.CONFIGS["beam32"]["steps"])
        log(f"[bench] beam32 frozen-field particle phase: {frozen['ms_per_step']} ms/step, "
            f"{frozen['roofline']['frac']} of HBM peak")
    ctx, cfg, mesh, parts, mi = setup(args.workload, args.particles)
    n_p = sum(p[2].size for p in parts.values())
    n_occ = int(np.unique(np.concatenate([p[2] for p in parts.values()])).size)
    if args.profile_steps is None:
        args.profile_steps = cfg.get("sort_every", 0) or 3
    solve = cfg["mode"] == "solve"
    sort_every = cfg.get("sort_every", 0)

    def prm_of(pc, solver):
        return qh.Context.step_params(field_mode=qh.FIELDS_SOLVE if solve else qh.FIELDS_FROZEN,
                                      precond=qh.PC_LEARNED if pc == "learned" else qh.PC_JACOBI,
                                      sort_every=sort_every, tol_edge=1e-8, tol_node=1e-8, max_it_edge=2000,
                                      max_it_node=5000, check_every=16,
                                      solver=qh.SOLVER_MIXED if solver == "mixed" else qh.SOLVER_FP64)

    def timed(prm, steps):
        t0 = time.perf_counter()
        ctx.pic_step(prm, steps, want_stats=False)   # returns after its stream is synchronised
        return time.perf_counter() - t0

    def profile(prm, steps):
        ctx.timing(True)
        pst = ctx.pic_step(prm, steps, want_stats=True)
        kt = ctx.timing_read()
        ctx.timing(False)
        kern = {}
        for k, (ms, cnt) in kt.items():
            if cnt:
                kern[k] = {"ms_total": round(ms, 4), "launches": cnt, "us_per_launch": round(1e3 * ms / cnt, 3)}
        return pst, kern

    def run(pc, solver):
        # a few untimed steps (the first solve of a configuration sizes its first check batch),
        # the timed steps, then a whole sort cycle with the two phase events per step only, and
        # one with a HIP event pair around every launch (per-kernel times; about 4 % slower)
        prm = prm_of(pc, solver)
        ctx.pic_step(prm, 2, want_stats=False)
        wall = timed(prm, args.steps)
        pst = ctx.pic_step(prm, args.profile_steps, want_stats=True)
        pst_k, kern = profile(prm, args.profile_steps)
        log(f"[bench] {pc} {solver}: {1e3 * wall / args.steps:.3f} ms/step, edge iters "
            f"{[s['edge_iters'] for s in pst]}, reliable updates {[s['edge_refinements'] for s in pst][:4]}")
        return {"wall": wall, "pst": pst, "pst_k": pst_k, "kernels": kern, "precond": pc, "solver": solver}

    st = ctx.pic_step(prm_of("jacobi", "fp64"), args.warmup, want_stats=True)
    log(f"[bench] warmup done: last step {st[-1]}")
    solvers = ["fp64", "mixed"] if solve else ["fp64"]
    runs = {f"jacobi_{sv}": run("jacobi", sv) for sv in solvers}
    train = None
    if solve and args.precond == "learned":
        # held-out (rhs, solution) pairs of the plain solver on this run (particle seed 0) validate
        # the network during training
        pairs = []
        for _ in range(2):
            ctx.pic_step(prm_of("jacobi", "fp64"), 1, want_stats=False)
            pairs.append(ctx.edge_system_download())
        rhs = np.stack([p[0] for p in pairs])
        sol = np.stack([p[1] for p in pairs])
        gen = None
        if args.pairs > 0:
            # training pairs: the plain solver's, recorded over the same workload with particle
            # seed 1 (its own context), the network trained there and carried over by save/load
            t0 = time.perf_counter()
            ctx1, _c1, _m1, _p1, _mi1 = setup(args.workload, args.particles, seed=1)
            if cfg["mode"] == "solve":
                ctx1.charge_background(1)
            ctx1.pairs_record(args.pairs)
            t1 = time.perf_counter()
            ctx1.pic_step(prm_of("jacobi", "fp64"), args.pairs, want_stats=False)
            gen = {"pairs": ctx1.pairs_count(), "seed": 1, "solver": "jacobi", "tol": 1e-8,
                   "s_generate": round(time.perf_counter() - t1, 2), "s_setup": round(t1 - t0, 2)}
            train = ctx1.precond_train(steps=args.train_steps, lr=3e-3, seed=1, validate_every=25, rhs=rhs, sol=sol,
                                       pair_weight=args.pair_weight)
            ctx.precond_load(ctx1.precond_save())
            ctx1.close()
            del ctx1
        else:
            train = ctx.precond_train(steps=args.train_steps, lr=3e-3, seed=1, validate_every=25, rhs=rhs, sol=sol)
        train["pair_weight"] = args.pair_weight if args.pairs > 0 else 0.0
        train["pair_generation"] = gen
        log(f"[bench] training: {train}")
        for sv in solvers:
            runs[f"learned_{sv}"] = run("learned", sv)
    headline = f"{args.precond if train else 'jacobi'}_{args.solver if solve else 'fp64'}"
    H = runs[headline]
    wall, pst, pst_k, kernels = H["wall"], H["pst"], H["pst_k"], H["kernels"]
    learned_used = H["precond"] == "learned"
    mixed_used = H["solver"] == "mixed"
    ms_step = 1e3 * wall / args.steps
    value = n_p * args.steps / wall
    crossings = float(np.mean([s["crossings"] for s in pst]))
    mi = ctx.mesh_info()  # now with the learned factor's sizes
    dom = max(kernels, key=lambda k: kernels[k]["ms_total"])

    def roof(k, kern, r):
        by = algorithmic_bytes(k, mi, n_p, crossings, learned=r["precond"] == "learned", mixed=r["solver"] == "mixed",
                               n_species=len(parts))
        if by is None or k not in kern:
            return None
        # the edge iterations' kernels: the time of all their launches over the iterations that
        # did work (launches past convergence return at once and are counted as part of it)
        its = sum(s["edge_iters"] for s in r["pst_k"])
        n_work = its if k in ("cg_spmv", "cg_update", "precond") and its else kern[k]["launches"]
        avg_s = kern[k]["ms_total"] / n_work * 1e-3
        ach = by / avg_s / 1e9
        hk = hip_kernels(k, r["solver"] == "mixed", r["precond"] == "learned")
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(k, args.workload, hk), "kernel": k,
                "hip_kernels": hk, "algorithmic_bytes_per_launch": int(by),
                "us_per_launch": round(avg_s * 1e6, 3), "working_launches": n_work}
    # the particle phase per step over a whole re-sort cycle (the sort is in), field prep, push,
    # walk, deposit, moves between blocks, sort; phase events only
    ms_part = float(np.mean([s["ms_particles"] for s in pst]))
    by_phase = phase_bytes(mi, n_p, crossings, n_occ)
    ach_phase = by_phase / (ms_part * 1e-3) / 1e9

    def per_iteration(kern, pst_):
        # edge CG cost per iteration: the kernels every iteration launches once (product, update,
        # and with the learned preconditioner its two passes), over the profiled iterations
        its = sum(s["edge_iters"] for s in pst_)
        if not its:
            return None
        parts_ = {k: round(1e3 * kern[k]["ms_total"] / its, 2) for k in ("cg_spmv", "cg_update", "precond")
                  if k in kern}
        return {"us_per_iteration": round(sum(parts_.values()), 2), "iterations": its, "us_by_kernel": parts_}

    def summary(r):
        return {"ms_per_step": round(1e3 * r["wall"] / args.steps, 4),
                "particle_steps_per_s": round(n_p * args.steps / r["wall"], 1),
                "field_solve_ms_per_step": round(float(np.mean([s["ms_fields"] for s in r["pst"]])), 4),
                "edge_iters": [s["edge_iters"] for s in r["pst"]],
                "edge_refinements": [s["edge_refinements"] for s in r["pst"]],
                "edge_res_max": max(s["edge_res"] for s in r["pst"]),
                "fallbacks": sum(s["fallbacks"] for s in r["pst"]),
                "edge_cg_iteration": per_iteration(r["kernels"], r["pst_k"])}
    out = {
        "metric": "particle-steps/s (gather+push+deposit), % HBM roofline; field-solve ms/step learned vs Jacobi",
        "value": round(value, 1), "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 push / int64 deposit / f64 edge residual" + (" with f32 PCG iterations" if mixed_used else " and PCG"),
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "particles": n_p,
                   "tets": mi.n_tets, "edges": mi.n_edges, "nnz_edge": mi.nnz_edge, "dt": cfg["dt"],
                   "sort_every": sort_every, "tol": 1e-8, "precond": H["precond"], "solver": H["solver"]},
        "roofline": roof(dom, kernels, H),
        "particle_phase": {"ms_per_step": round(ms_part, 4),
                           "particle_steps_per_s": round(n_p / (ms_part * 1e-3), 1),
                           "steps_timed": len(pst), "sort_every": sort_every,
                           "covers": "field prep, gather/push/walk/deposit, moves between blocks, the sort "
                                     "once per cycle (HIP events around the phase, every step of the cycle)",
                           "roofline": {"bound": "hbm", "achieved": round(ach_phase, 1), "peak": HBM_PEAK_GBS,
                                        "unit": "GB/s", "frac": round(ach_phase / HBM_PEAK_GBS, 4),
                                        "algorithmic_bytes_per_step": int(by_phase), "occupied_tets": n_occ,
                                        "crossings_per_step": crossings}},
        "particle_kernels": roof("particle_step", kernels, H),
        "field_solve_ms_per_step": {k: summary(r)["field_solve_ms_per_step"] for k, r in runs.items()},
        "solvers": {k: summary(r) for k, r in runs.items()},
        "solver": {"edge_iters": [s["edge_iters"] for s in pst], "node_iters": [s["node_iters"] for s in pst],
                   "edge_res": max(s["edge_res"] for s in pst), "gauss_res": max(s["gauss_res"] for s in pst),
                   "gauss_res_rho": max(s["gauss_res_rho"] for s in pst),
                   "fallbacks": sum(s["fallbacks"] for s in pst)},
        "kernels": kernels,
        "crossings_per_step": crossings,
        "foreign_deposits_per_step": float(np.mean([s["foreign"] for s in pst])),
    }
    if train:
        out["learned_training"] = train
    if frozen:
        out["frozen_particle_phase"] = frozen
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        try:
            out["cpu_baseline"] = cpu_baseline(args.workload, cfg, mesh, parts, args.cpu_sample)
        except Exception as ex:  # the baseline must not hide the GPU result
            out["cpu_baseline"] = {"error": repr(ex)}
        log(f"[bench] cpu baseline {time.perf_counter() - t0:.1f}s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
