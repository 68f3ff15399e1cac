"""Host code under AddressSanitizer (CPU; no GPU calls): the library's host C++ (mesh complex,
FP64 assembly, the explicit-limit pass, topology and matrix copies, argument checks) and the
oracle's C particle walk, each built with the sanitizer and run in a child process with its
runtime preloaded. Any invalid access aborts the child with a report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r"""
import ctypes
ctypes.CDLL(None).__asan_init          # the preloaded runtime is live in this process
"""

LIBRARY_RUN = PROBE + r"""
import numpy as np
import paper_2103_06737_amd as qh
import qh_inputs as qi
assert qh.LIB_PATH.endswith("libqh_asan.so"), qh.LIB_PATH
for m in (qi.make_mesh(qi.CONFIGS["jitter4"]), qi.BoxMesh(6), qi.CylinderMesh(0.02, 0.1, 4, 6),
          qi.make_mesh(dict(qi.CONFIGS["graded96"], n=8))):
    for bc in (qh.BC_PEC, qh.BC_NEUMANN):
        ctx = qh.Context(-1)
        ctx.set_boundary(bc)
        ctx.mesh_upload(m.xyz, m.tets)
        ctx.set_physics(qi.EPS0, qi.MU0, 1e-11, 1.0, 2.0 ** -56)
        info = ctx.mesh_info()
        assert info.dt_cfl > 0
        topo = ctx.topology()
        for which in range(6):
            ctx.matrix(which)
        for call in (lambda: ctx.precond_load(b"QHPRECND" + bytes(60)), lambda: ctx.set_walls(7)):
            try:
                call()
            except qh.QhError:
                pass
        ctx.close()
bad = qi.BoxMesh(2)
t = bad.tets.copy()
t[0, 0] = 10 ** 6
try:
    qh.Context(-1).mesh_upload(bad.xyz, t)
except qh.QhError:
    pass
print("library host code clean")
"""

ORACLE_RUN = PROBE + r"""
import numpy as np
import qh_inputs as qi
from oracle import particles
from oracle.complex_ import Complex
from oracle.particles import ParticleOracle
from oracle.whitney import Operators
assert particles.LIB.endswith("liborc_asan.so")
for m, absorb in ((qi.make_mesh(qi.CONFIGS["jitter4"]), False), (qi.CylinderMesh(0.02, 0.1, 4, 6), True)):
    cx = Complex(m.xyz, m.tets)
    op = Operators(cx, qi.EPS0, qi.MU0)
    po = ParticleOracle(cx, op.Minv)
    rng = np.random.default_rng(0)
    t = rng.integers(cx.Nt, size=300)
    lam = rng.dirichlet(np.ones(4), size=300)
    x = np.einsum("pi,pij->pj", lam, cx.xyz[cx.tets[t]])
    v = rng.standard_normal((300, 3)) * 3e8
    e = rng.standard_normal(cx.Ne) * 1e3
    out = po.push(e, np.zeros(cx.Nf), x, v, t, -1.76e11, 1e-10, -1, dump_segments=20000, absorb=absorb)
    s = out["segments"]
    po.deposit_list(s["tet"], s["l0"], s["l1"], -np.ones(len(s["tet"])), out["tet"][~out["absorbed"]],
                    po.quantize_points(out["x"][~out["absorbed"]], out["tet"][~out["absorbed"]]),
                    -np.ones(int((~out["absorbed"]).sum())))
    po.gather(e, np.zeros(cx.Nf), x, t)
print("oracle walk clean")
"""


def _instrumented(lib):
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    return "__asan_report" in syms


def _run(code, env_extra):
    env = dict(os.environ, **env_extra, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stderr[-4000:]
    return r.stdout


def test_library_host_code_under_asan():
    from tests import asan_build
    lib = asan_build.build_library()
    assert _instrumented(lib)
    out = _run(LIBRARY_RUN, {"QH_LIBQH": lib, "LD_PRELOAD": asan_build.runtime("clang")})
    assert "library host code clean" in out


def test_oracle_walk_under_asan():
    from tests import asan_build
    lib = asan_build.build_oracle()
    assert _instrumented(lib)
    out = _run(ORACLE_RUN, {"QH_ORC_LIB": lib, "LD_PRELOAD": asan_build.runtime("gcc")})
    assert "oracle walk clean" in out
