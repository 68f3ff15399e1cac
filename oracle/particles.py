"""ctypes front of the FP64 particle oracle in pic.c (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from .complex_ import Complex

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic.c")
LIB = os.environ.get("QH_ORC_LIB") or os.path.join(HERE, "_build", "liborc.so")  # QH_ORC_LIB: another build
F_BITS = 20


def build(force: bool = True) -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Mesh(C.Structure):
    _fields_ = [("Nn", C.c_int64), ("Ne", C.c_int64), ("Nf", C.c_int64), ("Nt", C.c_int64),
                ("tet_nodes", C.c_void_p), ("tet_edges", C.c_void_p), ("tet_faces", C.c_void_p),
                ("tet_nbr", C.c_void_p), ("minv", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        p = C.c_void_p
        L.orc_push.restype = C.c_int64
        L.orc_push.argtypes = [p, p, p, C.c_int64, p, p, p, C.c_double, C.c_double, C.c_int64,
                               C.c_int, C.c_int, C.c_int, p, p, p, p, C.c_int64, p, p, p, p, p, C.c_int]
        L.orc_deposit_list.restype = None
        L.orc_deposit_list.argtypes = [p, C.c_int64, p, p, p, p, C.c_int64, p, p, p, C.c_int, p, p]
        L.orc_quantize_points.argtypes = [p, C.c_int64, p, p, C.c_int, p]
        L.orc_gather.argtypes = [p, p, p, C.c_int64, p, p, p, p]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class ParticleOracle:
    """Holds contiguous FP64/int64 copies of the mesh arrays the C oracle reads."""

    def __init__(self, cx: Complex, Minv: np.ndarray):
        self.cx = cx
        self.arrs = dict(
            tet_nodes=np.ascontiguousarray(cx.tets, dtype=np.int64),
            tet_edges=np.ascontiguousarray(cx.tet_edges, dtype=np.int64),
            tet_faces=np.ascontiguousarray(cx.tet_faces, dtype=np.int64),
            tet_nbr=np.ascontiguousarray(cx.tet_nbr, dtype=np.int64),
            minv=np.ascontiguousarray(Minv, dtype=np.float64).reshape(-1),
        )
        a = self.arrs
        self.m = _Mesh(cx.Nn, cx.Ne, cx.Nf, cx.Nt, _ptr(a["tet_nodes"]), _ptr(a["tet_edges"]),
                       _ptr(a["tet_faces"]), _ptr(a["tet_nbr"]), _ptr(a["minv"]))

    def push(self, e, b_real, x, v, tet, qm, dt, z, g=None, Q=None, max_seg=64,
             dump_segments=0, nthreads=0, absorb=False):
        """Advance particles one step (in place on float64 copies that are returned). absorb:
        walls absorb (a particle stops at the wall point, lost_flags 2, and its charge is not
        deposited) instead of reflecting."""
        x = np.ascontiguousarray(x, dtype=np.float64).copy()
        v = np.ascontiguousarray(v, dtype=np.float64).copy()
        tet = np.ascontiguousarray(tet, dtype=np.int64).copy()
        n = tet.shape[0]
        g = np.zeros(self.cx.Ne, np.int64) if g is None else g
        Q = np.zeros(self.cx.Nn, np.int64) if Q is None else Q
        lost = np.zeros(n, np.int32)
        stats = np.zeros(2, np.int64)
        seg = None
        cnt = np.zeros(1, np.int64)
        if dump_segments:
            cap = int(dump_segments)
            seg = dict(tet=np.zeros(cap, np.int64), l0=np.zeros((cap, 4), np.int64),
                       l1=np.zeros((cap, 4), np.int64), pid=np.zeros(cap, np.int64))
        e = np.ascontiguousarray(e, dtype=np.float64)
        b_real = np.ascontiguousarray(b_real, dtype=np.float64)
        nl = lib().orc_push(C.byref(self.m), _ptr(e), _ptr(b_real), n, _ptr(x), _ptr(v), _ptr(tet),
                            float(qm), float(dt), int(z), F_BITS, int(max_seg), int(bool(absorb)), _ptr(g), _ptr(Q),
                            _ptr(lost), _ptr(stats), int(dump_segments), _ptr(cnt),
                            _ptr(seg["tet"]) if seg else None, _ptr(seg["l0"]) if seg else None,
                            _ptr(seg["l1"]) if seg else None, _ptr(seg["pid"]) if seg else None,
                            int(nthreads))
        out = dict(x=x.reshape(-1, 3), v=v.reshape(-1, 3), tet=tet, g=g, Q=Q, lost=int(nl),
                   lost_flags=lost, absorbed=lost == 2, crossings=int(stats[0]), wall_hits=int(stats[1]))
        if seg:
            k = int(cnt[0])
            out["segments"] = {kk: vv[:k] for kk, vv in seg.items()}
        return out

    def deposit_list(self, seg_tet, l0, l1, seg_z, pt_tet, pt_l, pt_z):
        g = np.zeros(self.cx.Ne, np.int64)
        Q = np.zeros(self.cx.Nn, np.int64)
        st = np.ascontiguousarray(seg_tet, np.int64)
        a0 = np.ascontiguousarray(l0, np.int64)
        a1 = np.ascontiguousarray(l1, np.int64)
        sz = np.ascontiguousarray(seg_z, np.int64)
        pt = np.ascontiguousarray(pt_tet, np.int64)
        pl = np.ascontiguousarray(pt_l, np.int64)
        pz = np.ascontiguousarray(pt_z, np.int64)
        lib().orc_deposit_list(C.byref(self.m), st.shape[0], _ptr(st), _ptr(a0), _ptr(a1), _ptr(sz),
                               pt.shape[0], _ptr(pt), _ptr(pl), _ptr(pz), F_BITS, _ptr(g), _ptr(Q))
        return g, Q

    def quantize_points(self, x, tet):
        x = np.ascontiguousarray(x, np.float64)
        t = np.ascontiguousarray(tet, np.int64)
        L = np.zeros((t.shape[0], 4), np.int64)
        lib().orc_quantize_points(C.byref(self.m), t.shape[0], _ptr(x), _ptr(t), F_BITS, _ptr(L))
        return L

    def gather(self, e, b_real, x, tet):
        x = np.ascontiguousarray(x, np.float64)
        t = np.ascontiguousarray(tet, np.int64)
        E = np.zeros((t.shape[0], 3))
        B = np.zeros((t.shape[0], 3))
        lib().orc_gather(C.byref(self.m), _ptr(np.ascontiguousarray(e, np.float64)),
                         _ptr(np.ascontiguousarray(b_real, np.float64)), t.shape[0], _ptr(x),
                         _ptr(t), _ptr(E), _ptr(B))
        return E, B
