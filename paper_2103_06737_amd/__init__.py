"""Python binding of libqh (argument marshalling only).

Every step of the PIC cycle runs in the HIP kernels of libqh.so; this module converts
numpy arrays to pointers and status codes to exceptions. The library must have been
built in-tree (``python -m paper_2103_06737_amd.build``); importing fails loudly
otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("QH_LIBQH") or os.path.join(HERE, "libqh.so")  # QH_LIBQH: another build (sanitizer tests)

QH_OK, QH_EINVAL, QH_ENOMEM, QH_EHIP, QH_ENOTCONV, QH_EOVERFLOW, QH_ELOST, QH_ESTATE, QH_EVERIFY = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
FIELDS_FROZEN, FIELDS_SOLVE, FIELDS_WAVE = 0, 1, 2
BC_PEC, BC_NEUMANN = 0, 1
WALLS_REFLECT, WALLS_ABSORB = 0, 1
PC_JACOBI, PC_LEARNED = 0, 1
SOLVER_FP64, SOLVER_MIXED = 0, 1
SYS_EDGE, SYS_NODE = 0, 1
KERNELS = ["field_prep", "particle_step", "sort", "edge_rhs", "cg_spmv", "cg_update", "cg_init",
           "gauss", "faraday", "true_res", "node_spmv", "node_update", "precond", "boundary"]
MLP_NPARAM = 5313
F_BITS = 20
EXPORTS = ["qh_create", "qh_destroy", "qh_last_error", "qh_mesh_upload", "qh_mesh_info",
           "qh_mesh_topology", "qh_set_physics", "qh_fields_upload", "qh_fields_download",
           "qh_fields_init_synthetic", "qh_species_add", "qh_particles_upload",
           "qh_particles_download", "qh_charge_background", "qh_pic_step", "qh_deposits_download",
           "qh_capture_segments", "qh_segments_download", "qh_deposit", "qh_field_solve",
           "qh_matrix_info", "qh_matrix_download", "qh_timing_enable", "qh_timing_read",
           "qh_precond_set_weights", "qh_precond_get_weights", "qh_precond_factor", "qh_precond_loss_grad",
           "qh_precond_train", "qh_edge_system_download", "qh_set_boundary", "qh_set_plane_wave",
           "qh_particles_count", "qh_particles_ids", "qh_set_walls", "qh_particles_inject", "qh_probe_fields",
           "qh_fields_decompose", "qh_locate", "qh_precond_save", "qh_precond_load", "qh_fields_upload_dev",
           "qh_fields_download_dev", "qh_deposits_download_dev", "qh_state_save", "qh_state_load",
           "qh_fields_energy", "qh_precond_apply", "qh_deposit_noalloc", "qh_pairs_record", "qh_pairs_count",
           "qh_pairs_add", "qh_precond_pair_loss_grad"]


class QhError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libqh error {code}: {msg}")
        self.code = code


class MeshInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_edges", C.c_int64), ("n_faces", C.c_int64),
                ("n_tets", C.c_int64), ("n_int_nodes", C.c_int64), ("n_int_edges", C.c_int64),
                ("nnz_edge", C.c_int64), ("nnz_node", C.c_int64), ("nnz_edge_c16", C.c_int64),
                ("nnz_factor", C.c_int64), ("nnz_factor_c16", C.c_int64), ("dt_cfl", C.c_double)]


class Phys(C.Structure):
    _fields_ = [("eps0", C.c_double), ("mu0", C.c_double), ("dt", C.c_double),
                ("u_q", C.c_double), ("u_b", C.c_double)]


class StepParams(C.Structure):
    _fields_ = [("field_mode", C.c_int32), ("sort_every", C.c_int32), ("precond", C.c_int32),
                ("gauss", C.c_int32), ("tol_edge", C.c_double), ("tol_node", C.c_double),
                ("max_it_edge", C.c_int32), ("max_it_node", C.c_int32),
                ("check_every", C.c_int32), ("verify", C.c_int32), ("solver", C.c_int32)]


class StepStats(C.Structure):
    _fields_ = [("edge_iters", C.c_int32), ("node_iters", C.c_int32), ("edge_res", C.c_double),
                ("node_res", C.c_double), ("gauss_res", C.c_double), ("crossings", C.c_int64),
                ("wall_hits", C.c_int64), ("lost", C.c_int64), ("continuity_bad", C.c_int64),
                ("divb_bad", C.c_int64), ("fallbacks", C.c_int32), ("ms_particles", C.c_float),
                ("ms_fields", C.c_float), ("foreign", C.c_int64), ("gauss_res_rho", C.c_double),
                ("edge_refinements", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrainParams(C.Structure):
    _fields_ = [("steps", C.c_int32), ("lr", C.c_float), ("seed", C.c_uint64), ("validate_every", C.c_int32),
                ("val_tol", C.c_double), ("val_max_it", C.c_int32), ("pair_weight", C.c_double)]


class TrainStats(C.Structure):
    _fields_ = [("steps_done", C.c_int32), ("loss_first", C.c_double), ("loss_last", C.c_double),
                ("val_iters_jacobi", C.c_int32), ("val_iters_best", C.c_int32), ("best_step", C.c_int32),
                ("ms", C.c_float), ("pair_loss_first", C.c_double), ("pair_loss_last", C.c_double),
                ("val_energy_err", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("res", C.c_double), ("fallback", C.c_int32), ("ms", C.c_float)]


_lib = None


def lib():
    """Load libqh.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2103_06737_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        p, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "qh_create": [C.POINTER(p), C.c_int, p],
            "qh_destroy": [p],
            "qh_mesh_upload": [p, i64, p, i64, p],
            "qh_set_boundary": [p, i32],
            "qh_set_plane_wave": [p, d, d, d, d],
            "qh_mesh_info": [p, C.POINTER(MeshInfo)],
            "qh_mesh_topology": [p, p, p, p, p, p, p, p, p],
            "qh_set_physics": [p, C.POINTER(Phys)],
            "qh_fields_upload": [p, p, p],
            "qh_fields_download": [p, p, p],
            "qh_fields_init_synthetic": [p, p, p, d, d, d],
            "qh_species_add": [p, d, i32, C.POINTER(i32)],
            "qh_particles_upload": [p, i32, i64, p, p, p],
            "qh_particles_download": [p, i32, p, p, p],
            "qh_particles_count": [p, i32, C.POINTER(i64)],
            "qh_particles_ids": [p, i32, p],
            "qh_set_walls": [p, i32],
            "qh_particles_inject": [p, i32, i64, p, p, p],
            "qh_probe_fields": [p, i64, p, p, p, p],
            "qh_fields_decompose": [p, d, i32, p, p, p, C.POINTER(SolveStats)],
            "qh_fields_energy": [p, p, p],
            "qh_locate": [p, i64, p, p],
            "qh_fields_upload_dev": [p, p, p],
            "qh_fields_download_dev": [p, p, p],
            "qh_deposits_download_dev": [p, p, p],
            "qh_precond_save": [p, p, C.POINTER(C.c_size_t)],
            "qh_state_save": [p, p, C.POINTER(C.c_size_t)],
            "qh_state_load": [p, p, C.c_size_t],
            "qh_precond_load": [p, p, C.c_size_t],
            "qh_charge_background": [p, i32],
            "qh_pic_step": [p, C.POINTER(StepParams), i32, p],
            "qh_deposits_download": [p, p, p],
            "qh_capture_segments": [p, i64],
            "qh_segments_download": [p, C.POINTER(i64), p, p, p, p, p, p],
            "qh_deposit": [p, i64, p, p, p, p, i64, p, p, p, p, p],
            "qh_deposit_noalloc": [p, i64, p, p, p, p, i64, p, p, p, p, p],
            "qh_field_solve": [p, i32, p, p, d, i32, i32, i32, C.POINTER(SolveStats)],
            "qh_matrix_info": [p, i32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)],
            "qh_matrix_download": [p, i32, p, p, p],
            "qh_timing_enable": [p, i32],
            "qh_timing_read": [p, i32, p, p],
            "qh_edge_system_download": [p, p, p],
            "qh_precond_set_weights": [p, p, i64],
            "qh_precond_get_weights": [p, p, i64],
            "qh_precond_factor": [p, C.POINTER(i64), p, p, p],
            "qh_precond_apply": [p, p, p],
            "qh_pairs_record": [p, i32],
            "qh_pairs_count": [p, C.POINTER(i32)],
            "qh_pairs_add": [p, i32, p, p],
            "qh_precond_pair_loss_grad": [p, p, C.POINTER(d), p],
            "qh_precond_loss_grad": [p, p, C.POINTER(d), p],
            "qh_precond_train": [p, C.POINTER(TrainParams), i32, p, p, C.POINTER(TrainStats)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None if name == "qh_destroy" else C.c_int
        L.qh_last_error.argtypes = [p]
        L.qh_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Context:
    """One libqh context (one mesh, its fields and particle species) on one device.

    device < 0 gives a host-only context (mesh build and assembly only)."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self.L = lib()
        h = C.c_void_p()
        rc = self.L.qh_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None)
        if rc != QH_OK:
            raise QhError(rc, "qh_create failed (no HIP device?)")
        self.h = h
        self.info = None

    def close(self):
        if self.h:
            self.L.qh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != QH_OK and rc not in allow:
            raise QhError(rc, self.L.qh_last_error(self.h).decode())
        return rc

    # mesh -----------------------------------------------------------------------------
    def set_boundary(self, mode):
        """BC_PEC (default) or BC_NEUMANN; before mesh_upload."""
        self._check(self.L.qh_set_boundary(self.h, int(mode)))

    def set_plane_wave(self, E0, f0, bandwidth, t0):
        """Plane wave through the natural boundary (E along -z, travelling along +x)."""
        self._check(self.L.qh_set_plane_wave(self.h, float(E0), float(f0), float(bandwidth), float(t0)))

    def mesh_upload(self, xyz, tets):
        xyz = _c(xyz, np.float64)
        tets = _c(tets, np.int32)
        self._check(self.L.qh_mesh_upload(self.h, xyz.shape[0], _ptr(xyz), tets.shape[0], _ptr(tets)))
        mi = MeshInfo()
        self._check(self.L.qh_mesh_info(self.h, C.byref(mi)))
        self.info = mi
        return mi

    def mesh_info(self):
        mi = MeshInfo()
        self._check(self.L.qh_mesh_info(self.h, C.byref(mi)))
        self.info = mi
        return mi

    def topology(self):
        mi = self.info
        out = dict(edges=np.zeros((mi.n_edges, 2), np.int32), faces=np.zeros((mi.n_faces, 3), np.int32),
                   tet_nodes=np.zeros((mi.n_tets, 4), np.int32), tet_edges=np.zeros((mi.n_tets, 6), np.int32),
                   tet_faces=np.zeros((mi.n_tets, 4), np.int32), tet_nbr=np.zeros((mi.n_tets, 4), np.int32),
                   wall_edge=np.zeros(mi.n_edges, np.uint8), wall_node=np.zeros(mi.n_nodes, np.uint8))
        self._check(self.L.qh_mesh_topology(self.h, *[_ptr(out[k]) for k in
                                                      ("edges", "faces", "tet_nodes", "tet_edges", "tet_faces",
                                                       "tet_nbr", "wall_edge", "wall_node")]))
        return out

    def set_physics(self, eps0, mu0, dt, u_q, u_b):
        self.phys = Phys(eps0, mu0, dt, u_q, u_b)
        self._check(self.L.qh_set_physics(self.h, C.byref(self.phys)))

    def matrix(self, which):
        import scipy.sparse as sp
        nr, nc, nz = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.L.qh_matrix_info(self.h, which, C.byref(nr), C.byref(nc), C.byref(nz)))
        ptr = np.zeros(nr.value + 1, np.int32)
        col = np.zeros(nz.value, np.int32)
        val = np.zeros(nz.value, np.float64)
        self._check(self.L.qh_matrix_download(self.h, which, _ptr(ptr), _ptr(col), _ptr(val)))
        return sp.csr_matrix((val, col, ptr), shape=(nr.value, nc.value))

    # fields ---------------------------------------------------------------------------
    def fields_upload(self, e, b):
        e = _c(e, np.float64)
        b = _c(b, np.int64)
        self._check(self.L.qh_fields_upload(self.h, _ptr(e), _ptr(b)))

    def fields_download(self):
        e = np.zeros(self.info.n_edges)
        b = np.zeros(self.info.n_faces, np.int64)
        self._check(self.L.qh_fields_download(self.h, _ptr(e), _ptr(b)))
        return e, b

    def fields_init_synthetic(self, white_e, white_a, sigma_e, bz, sigma_b):
        we = _c(white_e, np.float64)
        wa = _c(white_a, np.float64)
        self._check(self.L.qh_fields_init_synthetic(self.h, _ptr(we), _ptr(wa), sigma_e, bz, sigma_b))

    # particles ------------------------------------------------------------------------
    def species_add(self, q_over_m, charge_number):
        sid = C.c_int32()
        self._check(self.L.qh_species_add(self.h, float(q_over_m), int(charge_number), C.byref(sid)))
        return sid.value

    def particles_upload(self, sid, x, v, tet=None):
        """tet None: the library locates the particles on the device."""
        x = _c(x, np.float32)
        v = _c(v, np.float32)
        tet = None if tet is None else _c(tet, np.int32)
        self._check(self.L.qh_particles_upload(self.h, sid, x.shape[0], _ptr(x), _ptr(v), _ptr(tet)))

    def particles_inject(self, sid, x, v, tet=None):
        """Append particles (ids continue); their charge is added to the present node charge."""
        x = _c(x, np.float32)
        v = _c(v, np.float32)
        tet = None if tet is None else _c(tet, np.int32)
        self._check(self.L.qh_particles_inject(self.h, sid, x.shape[0], _ptr(x), _ptr(v), _ptr(tet)))

    # device pointers (e.g. torch tensors' data_ptr()), ordered on the context's stream
    def fields_upload_dev(self, e_ptr, b_ptr):
        self._check(self.L.qh_fields_upload_dev(self.h, C.c_void_p(e_ptr), C.c_void_p(b_ptr)))

    def fields_download_dev(self, e_ptr, b_ptr):
        self._check(self.L.qh_fields_download_dev(self.h, C.c_void_p(e_ptr) if e_ptr else None,
                                                  C.c_void_p(b_ptr) if b_ptr else None))

    def deposits_download_dev(self, g_ptr, q_ptr):
        self._check(self.L.qh_deposits_download_dev(self.h, C.c_void_p(g_ptr) if g_ptr else None,
                                                    C.c_void_p(q_ptr) if q_ptr else None))

    def locate(self, xyz):
        """Tet holding each point (-1 outside the mesh), found on the device."""
        xyz = _c(xyz, np.float64)
        tet = np.zeros(xyz.shape[0], np.int32)
        self._check(self.L.qh_locate(self.h, xyz.shape[0], _ptr(xyz), _ptr(tet)))
        return tet

    def particles_count(self, sid):
        n = C.c_int64()
        self._check(self.L.qh_particles_count(self.h, sid, C.byref(n)))
        return n.value

    def particles_ids(self, sid):
        ids = np.zeros(self.particles_count(sid), np.int32)
        self._check(self.L.qh_particles_ids(self.h, sid, _ptr(ids)))
        return ids

    def particles_download(self, sid):
        """(x, v, tet) ordered by particle id (see particles_ids)."""
        n = self.particles_count(sid)
        x = np.zeros((n, 3), np.float32)
        v = np.zeros((n, 3), np.float32)
        t = np.zeros(n, np.int32)
        self._check(self.L.qh_particles_download(self.h, sid, _ptr(x), _ptr(v), _ptr(t)))
        return x, v, t

    def set_walls(self, mode):
        """WALLS_REFLECT (default) or WALLS_ABSORB."""
        self._check(self.L.qh_set_walls(self.h, int(mode)))

    def probe_fields(self, xyz, tet):
        """E (V/m) and B (T) at points (FP32 evaluation from the present e and b)."""
        xyz = _c(xyz, np.float64)
        tet = _c(tet, np.int32)
        E = np.zeros((tet.shape[0], 3))
        B = np.zeros((tet.shape[0], 3))
        self._check(self.L.qh_probe_fields(self.h, tet.shape[0], _ptr(xyz), _ptr(tet), _ptr(E), _ptr(B)))
        return E, B

    def charge_background(self, mode):
        self._check(self.L.qh_charge_background(self.h, int(mode)))

    # cycle ----------------------------------------------------------------------------
    @staticmethod
    def step_params(field_mode=FIELDS_FROZEN, sort_every=0, precond=PC_JACOBI, gauss=1,
                    tol_edge=1e-8, tol_node=1e-8, max_it_edge=2000, max_it_node=5000,
                    check_every=8, verify=0, solver=0):
        return StepParams(field_mode, sort_every, precond, gauss, tol_edge, tol_node, max_it_edge,
                          max_it_node, check_every, verify, solver)

    def pic_step(self, params, n_steps=1, want_stats=True, allow=()):
        stats = (StepStats * n_steps)() if want_stats else None
        rc = self.L.qh_pic_step(self.h, C.byref(params), int(n_steps),
                                C.cast(stats, C.c_void_p) if stats is not None else None)
        self._check(rc, allow)
        return [s.as_dict() for s in stats] if stats is not None else None

    def edge_system_download(self):
        n = self.info.n_int_edges
        rhs = np.zeros(n)
        sol = np.zeros(n)
        self._check(self.L.qh_edge_system_download(self.h, _ptr(rhs), _ptr(sol)))
        return rhs, sol

    def deposits_download(self):
        g = np.zeros(self.info.n_edges, np.int64)
        Q = np.zeros(self.info.n_nodes, np.int64)
        self._check(self.L.qh_deposits_download(self.h, _ptr(g), _ptr(Q)))
        return g, Q

    def capture_segments(self, cap):
        self._check(self.L.qh_capture_segments(self.h, int(cap)))
        self._cap = int(cap)

    def segments_download(self):
        cap = self._cap
        n = C.c_int64()
        out = dict(pid=np.zeros(cap, np.int32), species=np.zeros(cap, np.int32), seq=np.zeros(cap, np.int32),
                   tet=np.zeros(cap, np.int32), lam0=np.zeros((cap, 4), np.int32), lam1=np.zeros((cap, 4), np.int32))
        self._check(self.L.qh_segments_download(self.h, C.byref(n), *[_ptr(out[k]) for k in
                                                                       ("pid", "species", "seq", "tet", "lam0", "lam1")]))
        k = min(n.value, cap)
        return n.value, {kk: vv[:k] for kk, vv in out.items()}

    def deposit(self, seg_tet, lam0, lam1, seg_z, pt_tet, pt_lam, pt_z):
        a = [_c(seg_tet, np.int32), _c(lam0, np.int32), _c(lam1, np.int32), _c(seg_z, np.int32),
             _c(pt_tet, np.int32), _c(pt_lam, np.int32), _c(pt_z, np.int32)]
        g = np.zeros(self.info.n_edges, np.int64)
        Q = np.zeros(self.info.n_nodes, np.int64)
        self._check(self.L.qh_deposit(self.h, a[0].shape[0], _ptr(a[0]), _ptr(a[1]), _ptr(a[2]), _ptr(a[3]),
                                      a[4].shape[0], _ptr(a[4]), _ptr(a[5]), _ptr(a[6]), _ptr(g), _ptr(Q)))
        return g, Q

    def deposit_noalloc(self, seg_tet, lam0, lam1, seg_z, pt_tet, pt_lam, pt_z):
        """qh_deposit through the library's static scratch array (no device allocation)."""
        a = [_c(seg_tet, np.int32), _c(lam0, np.int32), _c(lam1, np.int32), _c(seg_z, np.int32),
             _c(pt_tet, np.int32), _c(pt_lam, np.int32), _c(pt_z, np.int32)]
        g = np.zeros(self.info.n_edges, np.int64)
        Q = np.zeros(self.info.n_nodes, np.int64)
        self._check(self.L.qh_deposit_noalloc(self.h, a[0].shape[0], _ptr(a[0]), _ptr(a[1]), _ptr(a[2]), _ptr(a[3]),
                                              a[4].shape[0], _ptr(a[4]), _ptr(a[5]), _ptr(a[6]), _ptr(g), _ptr(Q)))
        return g, Q

    def fields_decompose(self, tol=1e-10, max_it=5000, allow=()):
        """Quasi-Helmholtz split of the present e: (E_ns node coefficients, E_s edge values,
        rho_bar = G^T [*eps] e on the nodes, solve stats)."""
        mi = self.mesh_info()
        e_ns = np.zeros(mi.n_nodes)
        e_s = np.zeros(mi.n_edges)
        rho = np.zeros(mi.n_nodes)
        st = SolveStats()
        rc = self.L.qh_fields_decompose(self.h, float(tol), int(max_it), _ptr(e_ns), _ptr(e_s), _ptr(rho), C.byref(st))
        self._check(rc, allow)
        return e_ns, e_s, rho, dict(iters=st.iters, res=st.res, ms=st.ms)

    def fields_energy(self):
        """(electric, magnetic) energy of the present fields in joules (see qh_fields_energy)."""
        we, wm = C.c_double(0.0), C.c_double(0.0)
        self._check(self.L.qh_fields_energy(self.h, C.byref(we), C.byref(wm)))
        return we.value, wm.value

    def field_solve(self, system, rhs, x0=None, tol=1e-8, max_it=5000, precond=PC_JACOBI, solver=SOLVER_FP64,
                    allow=()):
        rhs = _c(rhs, np.float64)
        x = np.zeros_like(rhs) if x0 is None else _c(x0, np.float64).copy()
        st = SolveStats()
        rc = self.L.qh_field_solve(self.h, int(system), _ptr(rhs), _ptr(x), float(tol), int(max_it),
                                   int(precond), int(solver), C.byref(st))
        self._check(rc, allow)
        return x, dict(iters=st.iters, res=st.res, fallback=st.fallback, ms=st.ms)

    # learned preconditioner -------------------------------------------------------------
    def state_save(self):
        """Checkpoint of the run as bytes (see qh_state_save)."""
        n = C.c_size_t(0)
        self._check(self.L.qh_state_save(self.h, None, C.byref(n)))
        buf = (C.c_ubyte * n.value)()
        self._check(self.L.qh_state_save(self.h, C.cast(buf, C.c_void_p), C.byref(n)))
        return bytes(buf)

    def state_load(self, blob):
        buf = (C.c_ubyte * len(blob)).from_buffer_copy(blob)
        self._check(self.L.qh_state_load(self.h, C.cast(buf, C.c_void_p), len(blob)))

    def precond_save(self):
        """The trained network as bytes (see qh_precond_save)."""
        n = C.c_size_t(0)
        self._check(self.L.qh_precond_save(self.h, None, C.byref(n)))
        buf = (C.c_ubyte * n.value)()
        self._check(self.L.qh_precond_save(self.h, C.cast(buf, C.c_void_p), C.byref(n)))
        return bytes(buf)

    def precond_load(self, blob):
        buf = (C.c_ubyte * len(blob)).from_buffer_copy(blob)
        self._check(self.L.qh_precond_load(self.h, C.cast(buf, C.c_void_p), len(blob)))

    def precond_set_weights(self, w):
        w = _c(w, np.float32)
        self._check(self.L.qh_precond_set_weights(self.h, _ptr(w), w.size))

    def precond_get_weights(self):
        w = np.zeros(MLP_NPARAM, np.float32)
        self._check(self.L.qh_precond_get_weights(self.h, _ptr(w), w.size))
        return w

    def precond_factor(self):
        nnz = C.c_int64()
        self._check(self.L.qh_precond_factor(self.h, C.byref(nnz), None, None, None))
        rows = np.zeros(nnz.value, np.int32)
        cols = np.zeros(nnz.value, np.int32)
        vals = np.zeros(nnz.value, np.float32)
        self._check(self.L.qh_precond_factor(self.h, C.byref(nnz), _ptr(rows), _ptr(cols), _ptr(vals)))
        return rows, cols, vals

    def precond_apply(self, r):
        """z = G^T (G r) with the current weights (the learned solve's application kernels)."""
        r = _c(r, np.float64)
        z = np.zeros_like(r)
        self._check(self.L.qh_precond_apply(self.h, _ptr(r), _ptr(z)))
        return z

    def precond_loss_grad(self, probes, want_grad=True):
        probes = _c(probes, np.float32)
        loss = C.c_double()
        grad = np.zeros(MLP_NPARAM, np.float32) if want_grad else None
        self._check(self.L.qh_precond_loss_grad(self.h, _ptr(probes), C.byref(loss), _ptr(grad)))
        return loss.value, grad

    def pairs_record(self, capacity):
        """Record the next field steps' (rhs, solution) pairs into a device bank of `capacity`."""
        self._check(self.L.qh_pairs_record(self.h, int(capacity)))

    def pairs_add(self, rhs, sol):
        rhs, sol = _c(rhs, np.float64), _c(sol, np.float64)
        self._check(self.L.qh_pairs_add(self.h, rhs.shape[0], _ptr(rhs), _ptr(sol)))

    def precond_pair_loss_grad(self, idx, want_grad=True):
        idx = _c(idx, np.int32)
        loss = C.c_double()
        grad = np.zeros(MLP_NPARAM, np.float32) if want_grad else None
        self._check(self.L.qh_precond_pair_loss_grad(self.h, _ptr(idx), C.byref(loss), _ptr(grad)))
        return loss.value, grad

    def pairs_count(self):
        n = C.c_int32()
        self._check(self.L.qh_pairs_count(self.h, C.byref(n)))
        return n.value

    def precond_train(self, steps=200, lr=3e-3, seed=1, validate_every=25, val_tol=1e-8, val_max_it=3000,
                      rhs=None, sol=None, pair_weight=0.0):
        P = TrainParams(steps, lr, seed, validate_every, val_tol, val_max_it, float(pair_weight))
        n_pairs = 0 if rhs is None else rhs.shape[0]
        rhs = None if rhs is None else _c(rhs, np.float64)
        sol = None if sol is None else _c(sol, np.float64)
        st = TrainStats()
        self._check(self.L.qh_precond_train(self.h, C.byref(P), n_pairs, _ptr(rhs), _ptr(sol), C.byref(st)))
        return st.as_dict()

    # timing ---------------------------------------------------------------------------
    def timing(self, on):
        self._check(self.L.qh_timing_enable(self.h, int(bool(on))))

    def timing_read(self):
        n = len(KERNELS)
        ms = np.zeros(n)
        cnt = np.zeros(n, np.int64)
        self._check(self.L.qh_timing_read(self.h, n, _ptr(ms), _ptr(cnt)))
        return {k: (ms[i], int(cnt[i])) for i, k in enumerate(KERNELS)}
