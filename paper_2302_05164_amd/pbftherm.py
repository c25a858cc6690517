"""Python binding of the pbftherm C ABI (include/pbftherm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libpbftherm.so.  PyTorch provides device memory (tensors) and the
stream (torch's current stream).  Importing this module fails loudly when the
library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbftherm.so")

PREC_FP64 = 64
PREC_FP32 = 32

_ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EMESH", -4: "EDEVICE", -5: "ENOCONV",
           -6: "ENONFINITE", -7: "ESTATE"}


class PbfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pbftherm {_ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Material(C.Structure):
    _fields_ = [("n_bp", C.c_int), ("T_bp", C.POINTER(C.c_double)), ("k_bp", C.POINTER(C.c_double)),
                ("cp_bp", C.POINTER(C.c_double)), ("rho", C.c_double), ("T_s", C.c_double),
                ("T_l", C.c_double), ("latent", C.c_double), ("powder_k_factor", C.c_double),
                ("powder_depth", C.c_double)]


class _Track(C.Structure):
    _fields_ = [("x0", C.c_double * 3), ("x1", C.c_double * 3), ("speed", C.c_double),
                ("power", C.c_double)]


class _SurfaceLoss(C.Structure):
    _fields_ = [("emissivity", C.c_double), ("T_inf", C.c_double), ("evap_on", C.c_int),
                ("T_v", C.c_double), ("C_P", C.c_double), ("C_T", C.c_double), ("C_M", C.c_double),
                ("h_v", C.c_double), ("T_h0", C.c_double), ("dT_max", C.c_double)]


class _Laser(C.Structure):
    _fields_ = [("kind", C.c_int), ("radius", C.c_double), ("absorptivity", C.c_double),
                ("h_powder", C.c_double), ("t_start", C.c_double), ("n_tracks", C.c_int),
                ("tracks", C.POINTER(_Track))]


class _Action(C.Structure):
    _fields_ = [("kind", C.c_int), ("step", C.c_int), ("slot", C.c_int)]


ACT_ADVANCE, ACT_STORE, ACT_RESTORE, ACT_TURN = 1, 2, 3, 4

_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)

# exported entry points and their argument types (also checked by the tests)
SIGNATURES = {
    "pbf_create": [C.POINTER(_vp)],
    "pbf_destroy": [_vp],
    "pbf_last_error": [_vp],
    "pbf_mesh_box": [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double],
    "pbf_mesh_info": [_vp, _i64p, _i64p, _i64p, _i64p, _i64p, _i64p],
    "pbf_set_dirichlet": [_vp, C.c_uint, C.c_double],
    "pbf_set_material": [_vp, C.POINTER(_Material)],
    "pbf_set_laser": [_vp, C.POINTER(_Laser)],
    "pbf_set_surface_loss": [_vp, C.POINTER(_SurfaceLoss)],
    "pbf_set_active_layers": [_vp, C.c_int],
    "pbf_active_info": [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int64), _dp],
    "pbf_activate_layers": [_vp, C.c_int, C.c_double, _vp, _vp, _vp],
    "pbf_set_track_powers": [_vp, _dp, C.c_double],
    "pbf_workspace_bytes": [_vp, C.POINTER(C.c_size_t)],
    "pbf_bind_device": [_vp, _vp, C.c_size_t, _vp],
    "pbf_init_state": [_vp, C.c_double, _vp, _vp, _vp],
    "pbf_explicit_steps": [_vp, _vp, _vp, _vp, C.c_double, C.c_double, C.c_int, C.c_int, _vp],
    "pbf_explicit_steps_noalloc": [_vp, _vp, _vp, _vp, C.c_double, C.c_double, C.c_int, C.c_int,
                                   C.POINTER(C.c_size_t), _vp],
    "pbf_assemble": [_vp, _vp, _vp, C.c_double, _vp, _vp, C.c_int, _vp],
    "pbf_stability_lambda": [_vp, _vp, C.c_int, _dp, _vp],
    "pbf_stability_dt": [_vp, _vp, C.c_int, _dp, _dp, _vp],
    "pbf_laplace_apply": [_vp, _vp, _vp, _vp],
    "pbf_set_implicit_preconditioner": [_vp, C.c_int, C.c_int, C.c_int],
    "pbf_set_newton_forcing": [_vp, C.c_int],
    "pbf_implicit_step": [_vp, _vp, _vp, _vp, C.c_double, C.c_double, C.c_double, C.c_int,
                          C.c_double, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _dp, _vp],
    "pbf_newton_work_bytes": [_vp, C.c_int, C.POINTER(C.c_size_t)],
    "pbf_implicit_step_newton": [_vp, _vp, _vp, _vp, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                 C.c_double, C.c_int, _vp, C.c_size_t, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                 C.POINTER(C.c_double), _vp],
    "pbf_set_probes": [_vp, C.c_int, _dp, _dp, _vp],
    "pbf_probe": [_vp, _vp, _vp, _vp],
    "pbf_objective": [_vp, _vp, _vp, _vp, _vp],
    "pbf_adjoint_step": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_double, C.c_double, _vp, _vp],
    "pbf_revolve_schedule": [C.c_int, C.c_int, C.POINTER(_Action), C.c_int, C.POINTER(C.c_int), _i64p],
    "pbf_adjoint_work_bytes": [_vp, C.c_int, C.POINTER(C.c_size_t)],
    "pbf_gradient_forward": [_vp, _vp, _vp, C.c_double, C.c_double, C.c_int, C.c_int, _vp, C.c_size_t,
                             _vp, _vp, _vp],
    "pbf_gradient_backward": [_vp, C.c_double, C.c_double, C.c_int, C.c_int, _vp, C.c_size_t, _vp, _vp,
                              _vp, _vp, _i64p, _vp],
    "pbf_energy": [_vp, _vp, _vp, _vp, C.c_double, C.c_double, _dp, _vp],
    "pbf_check_finite": [_vp, _vp, C.c_int64, C.POINTER(C.c_int), _dp, _vp],
    "pbf_mesh_octree": [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                        C.c_int, C.c_int64, C.POINTER(C.c_int32)],
    "pbf_octree_info": [_vp, _i64p, _i64p, C.POINTER(C.c_int)],
    "pbf_mesh_octree_growing": [_vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                C.c_int, C.c_int64, C.c_int64, C.POINTER(C.c_int32)],
    "pbf_octree_history_min": [_vp, _vp, _dp, _vp],
    "pbf_octree_layer_leaves": [_vp, _dp, C.c_int64, C.c_int64, C.c_double, C.POINTER(C.c_int32), C.c_int64,
                                _i64p],
    "pbf_octree_grow_bytes": [_vp, C.c_int64, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_size_t), _i64p,
                              _i64p],
    "pbf_octree_path_leaves": [_vp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int,
                               C.c_double, C.c_int, C.POINTER(_Track), C.c_double, C.c_double,
                               C.POINTER(C.c_int32), C.c_int64, _i64p],
    "pbf_octree_remesh_bytes": [_vp, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_size_t), _i64p, _i64p],
    "pbf_octree_remesh": [_vp, _vp, C.c_size_t, _vp, _vp, _vp, _vp, _vp],
    "pbf_dof_coords": [_vp, _dp],
    "pbf_timing_begin": [_vp, C.c_int, C.c_int],
    "pbf_timing_end": [_vp, _dp, _dp, _i64p],
}

_lib = None


def load_library(path: str = LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(hipcc, gfx950); there is no fallback implementation")
    L = C.CDLL(path)
    for name, args in SIGNATURES.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.pbf_last_error.restype = C.c_char_p
    L.pbf_destroy.restype = None
    _lib = L
    return L


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return C.c_void_p(t.data_ptr())


def _aligned(nbytes, device):
    """Device byte buffer with a 256-byte aligned start: (tensor, address)."""
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    base = buf.data_ptr()
    return buf, base + (-base) % 256


def _track_array(tracks):
    tr = np.asarray(tracks, dtype=np.float64).reshape(-1, 8)
    arr = (_Track * max(1, len(tr)))()
    for i, row in enumerate(tr):
        arr[i].x0[:] = row[0:3]
        arr[i].x1[:] = row[3:6]
        arr[i].speed = row[6]
        arr[i].power = row[7]
    return arr, len(tr)


def octree_path_leaves(nx, ny, nz, L, max_level, radius, tracks, s_lo, s_hi):
    """pbf_octree_path_leaves (host only): leaves (n, 4) int32 of the octree over
    nx x ny x nz coarse cells refined to max_level within `radius` of the scan
    path between arc lengths s_lo and s_hi, in Morton order."""
    lib = load_library()
    arr, nt = _track_array(tracks)
    n = C.c_int64(0)
    args = (None, int(nx), int(ny), int(nz), float(L[0]), float(L[1]), float(L[2]), int(max_level),
            float(radius), nt, arr, float(s_lo), float(s_hi))
    st = lib.pbf_octree_path_leaves(*args, None, 0, C.byref(n))
    if st != 0:
        raise PbfError(st, lib.pbf_last_error(None).decode())
    out = np.empty((n.value, 4), dtype=np.int32)
    st = lib.pbf_octree_path_leaves(*args, out.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n))
    if st != 0:
        raise PbfError(st, lib.pbf_last_error(None).decode())
    return out


def revolve_schedule(n_steps, n_snaps, with_actions=True):
    """Binomial checkpoint schedule (host only): (list of (kind, step, slot),
    number of forward steps)."""
    L = load_library()
    na, adv = C.c_int(0), C.c_int64(0)
    st = L.pbf_revolve_schedule(int(n_steps), int(n_snaps), None, 0, C.byref(na), C.byref(adv))
    if st != 0:
        raise PbfError(st, L.pbf_last_error(None).decode())
    if not with_actions:
        return None, adv.value
    arr = (_Action * max(1, na.value))()
    st = L.pbf_revolve_schedule(int(n_steps), int(n_snaps), arr, na.value, C.byref(na), C.byref(adv))
    if st != 0:
        raise PbfError(st, L.pbf_last_error(None).decode())
    return [(a.kind, a.step, a.slot) for a in arr[: na.value]], adv.value


def _f64(t, n, name):
    if t.dtype != torch.float64 or t.numel() != n:
        raise ValueError(f"{name}: expected {n} float64 values, got {t.numel()} {t.dtype}")
    return _ptr(t)


class Simulation:
    """One uniform-box problem bound to one GPU.  Set-up order: constructor (mesh),
    set_dirichlet, set_material, set_laser, bind(); then init_state() and the
    stepping calls.  State tensors (T, rc) belong to the caller."""

    def __init__(self, degree, nx, ny, nz, L, device="cuda:0", max_level=None, leaves=None, top=None):
        """Box mesh of nx*ny*nz cells, or (leaves given) an octree over those coarse
        cells with leaves (n, 4) = (level, ix, iy, iz); with `top` (finest cells)
        a growing octree whose active part is z < top."""
        self.lib = load_library()
        self.device = torch.device(device)
        self.ctx = _vp()
        self._check(self.lib.pbf_create(C.byref(self.ctx)), use_ctx=False)
        if leaves is None:
            self._check(self.lib.pbf_mesh_box(self.ctx, degree, nx, ny, nz, *map(float, L)))
        else:
            lv = np.ascontiguousarray(leaves, dtype=np.int32).reshape(-1, 4)
            if top is None:
                self._check(self.lib.pbf_mesh_octree(self.ctx, degree, nx, ny, nz, *map(float, L), int(max_level),
                                                     len(lv), lv.ctypes.data_as(C.POINTER(C.c_int32))))
            else:
                self._check(self.lib.pbf_mesh_octree_growing(self.ctx, degree, nx, ny, nz, *map(float, L),
                                                             int(max_level), int(top), len(lv),
                                                             lv.ctypes.data_as(C.POINTER(C.c_int32))))
        self.octree = leaves is not None
        self.workspace = None
        self.n_tracks = 0
        self.n_probes = 0

    def __del__(self):
        try:
            if getattr(self, "ctx", None) and self.ctx.value:
                self.lib.pbf_destroy(self.ctx)
                self.ctx = _vp()
        except TypeError:  # interpreter shutdown: ctypes already torn down
            pass

    def _check(self, st, use_ctx=True):
        if st != 0:
            msg = self.lib.pbf_last_error(self.ctx if use_ctx else None)
            raise PbfError(st, msg.decode() if msg else "")

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    # -- description ---------------------------------------------------------
    def info(self):
        v = [C.c_int64() for _ in range(6)]
        self._check(self.lib.pbf_mesh_info(self.ctx, *[C.byref(x) for x in v]))
        keys = ("n_dofs", "n_cells", "n_qp", "n_hist_layers", "n_hist_cells", "n_hist_qp")
        return dict(zip(keys, (x.value for x in v)))

    def set_dirichlet(self, face_mask, T_D):
        self._check(self.lib.pbf_set_dirichlet(self.ctx, int(face_mask), float(T_D)))

    def set_material(self, T_bp, k_bp, cp_bp, rho, T_s, T_l, latent, powder_k_factor,
                     powder_depth):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (T_bp, k_bp, cp_bp)]
        m = _Material(len(arrs[0]), *[a.ctypes.data_as(_dp) for a in arrs], float(rho),
                      float(T_s), float(T_l), float(latent), float(powder_k_factor),
                      float(powder_depth))
        self._check(self.lib.pbf_set_material(self.ctx, C.byref(m)))

    def set_laser(self, kind, radius, absorptivity, h_powder, t_start, tracks):
        arr, nt = _track_array(tracks)
        l = _Laser(int(kind), float(radius), float(absorptivity), float(h_powder), float(t_start), nt, arr)
        self._check(self.lib.pbf_set_laser(self.ctx, C.byref(l)))
        self.n_tracks = nt

    def set_surface_loss(self, emissivity=0.0, T_inf=293.0, evap_on=False, T_v=3000.0, C_P=54.0e3,
                         C_T=5.0e4, C_M=1.0e-3, h_v=6.0e6, T_h0=663.0, dT_max=1000.0):
        """Radiation and evaporation on the free top surface (off when emissivity
        is 0 and evap_on is False)."""
        r = _SurfaceLoss(float(emissivity), float(T_inf), 1 if evap_on else 0, float(T_v), float(C_P),
                         float(C_T), float(C_M), float(h_v), float(T_h0), float(dT_max))
        self._check(self.lib.pbf_set_surface_loss(self.ctx, C.byref(r)))

    def set_active_layers(self, nz_active):
        """Growing box: only the bottom nz_active cell layers are active (before bind)."""
        self._check(self.lib.pbf_set_active_layers(self.ctx, int(nz_active)))

    def active_info(self):
        nz, nd, lz = C.c_int(0), C.c_int64(0), C.c_double(0)
        self._check(self.lib.pbf_active_info(self.ctx, C.byref(nz), C.byref(nd), C.byref(lz)))
        return {"nz_active": nz.value, "n_active_dofs": nd.value, "Lz_active": lz.value}

    def activate_layers(self, nz_new, T0, T, rc):
        """Activate cell layers up to nz_new: new nodes start at T0, new cells as powder."""
        i = self.info()
        self._check(self.lib.pbf_activate_layers(self.ctx, int(nz_new), float(T0), _f64(T, i["n_dofs"], "T"),
                                                 _ptr(rc) if i["n_hist_qp"] else None, self._stream()))

    def set_track_powers(self, powers, absorptivity):
        p = np.ascontiguousarray(powers, dtype=np.float64)
        self._check(self.lib.pbf_set_track_powers(self.ctx, p.ctypes.data_as(_dp), float(absorptivity)))

    # -- device ------------------------------------------------------------------
    def bind(self):
        nb = C.c_size_t()
        self._check(self.lib.pbf_workspace_bytes(self.ctx, C.byref(nb)))
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._check(self.lib.pbf_bind_device(self.ctx, C.c_void_p(base + off), nb.value,
                                             self._stream()))

    def new_state(self):
        i = self.info()
        T = torch.empty(i["n_dofs"], dtype=torch.float64, device=self.device)
        rc = torch.empty(max(1, i["n_hist_qp"]), dtype=torch.float64, device=self.device)
        return T, rc

    def init_state(self, T0, T=None, rc=None):
        if T is None:
            T, rc = self.new_state()
        i = self.info()
        self._check(self.lib.pbf_init_state(self.ctx, float(T0), _f64(T, i["n_dofs"], "T"),
                                            _ptr(rc) if i["n_hist_qp"] else None, self._stream()))
        return T, rc

    def explicit_steps(self, T, rc, t0, dt, n_steps, precision=PREC_FP64, T_tmp=None):
        i = self.info()
        if T_tmp is None:
            T_tmp = torch.empty_like(T)
        self._check(self.lib.pbf_explicit_steps(
            self.ctx, _f64(T, i["n_dofs"], "T"), _f64(T_tmp, i["n_dofs"], "T_tmp"),
            _ptr(rc) if i["n_hist_qp"] else None, float(t0), float(dt), int(n_steps),
            int(precision), self._stream()))
        return T

    def explicit_steps_noalloc(self, T, rc, t0, dt, n_steps, T_tmp, precision=PREC_FP64):
        """pbf_explicit_steps_noalloc: the same steps with the scratch in the
        library's static device array (no workspace needed).  Returns the
        scratch bytes the mesh needs."""
        i = self.info()
        need = C.c_size_t(0)
        self._check(self.lib.pbf_explicit_steps_noalloc(
            self.ctx, _f64(T, i["n_dofs"], "T"), _f64(T_tmp, i["n_dofs"], "T_tmp"),
            _ptr(rc) if i["n_hist_qp"] else None, float(t0), float(dt), int(n_steps),
            int(precision), C.byref(need), self._stream()))
        return need.value

    def assemble(self, T, rc, t, precision=PREC_FP64):
        i = self.info()
        f = torch.empty_like(T)
        Cl = torch.empty_like(T)
        self._check(self.lib.pbf_assemble(self.ctx, _f64(T, i["n_dofs"], "T"),
                                          _ptr(rc) if i["n_hist_qp"] else None, float(t),
                                          _ptr(f), _ptr(Cl), int(precision), self._stream()))
        return f, Cl

    def stability_lambda(self, v0, iters):
        i = self.info()
        lam = C.c_double()
        self._check(self.lib.pbf_stability_lambda(self.ctx, _f64(v0, i["n_dofs"], "v0"), int(iters),
                                                  C.byref(lam), self._stream()))
        return lam.value

    def laplace_apply(self, x, y=None):
        """y = K x, the unit-conductivity Laplace operator (reference kernel)."""
        i = self.info()
        if y is None:
            y = torch.empty_like(x)
        self._check(self.lib.pbf_laplace_apply(self.ctx, _f64(x, i["n_dofs"], "x"), _f64(y, i["n_dofs"], "y"),
                                               self._stream()))
        return y

    def stability_dt(self, v0, iters):
        """Critical explicit step 2/lambda_max (eq. explicit_time_step)."""
        i = self.info()
        dt = C.c_double()
        self._check(self.lib.pbf_stability_dt(self.ctx, _f64(v0, i["n_dofs"], "v0"), int(iters),
                                              C.byref(dt), None, self._stream()))
        return dt.value

    def newton_work(self, restart=30):
        """Device buffer for implicit_step_newton with the given GMRES restart length."""
        nb = C.c_size_t()
        self._check(self.lib.pbf_newton_work_bytes(self.ctx, int(restart), C.byref(nb)))
        buf, addr = _aligned(nb.value, self.device)
        return {"buf": buf, "addr": addr, "bytes": nb.value, "restart": int(restart)}

    def implicit_step_newton(self, T_n, rc, t, dt, lin_rtol=1e-10, restart=30, lin_max_it=10000, newton_tol=1e-8,
                             newton_max_it=30, T_out=None, work=None, check=True):
        i = self.info()
        if work is None or work["restart"] != restart:
            work = self.newton_work(restart)
        if T_out is None:
            T_out = torch.empty_like(T_n)
        it, nit, res = C.c_int(0), C.c_int(0), C.c_double(0)
        st = self.lib.pbf_implicit_step_newton(
            self.ctx, _f64(T_n, i["n_dofs"], "T_n"), _f64(T_out, i["n_dofs"], "T_out"),
            _ptr(rc) if i["n_hist_qp"] else None, float(t), float(dt), float(lin_rtol), int(restart),
            int(lin_max_it), float(newton_tol), int(newton_max_it), C.c_void_p(work["addr"]), work["bytes"],
            C.byref(it), C.byref(nit), C.byref(res), self._stream())
        if check:
            self._check(st)
        return T_out, dict(status=st, lin_iters=it.value, newton_iters=nit.value, rel_res=res.value)

    def set_preconditioner(self, kind, smoothing_degree=2, coarse_degree=8):
        """pbf_set_implicit_preconditioner: 'jacobi' or 'multigrid'; rebinds the
        workspace (the multigrid levels take memory from it)."""
        k = {"jacobi": 0, "multigrid": 1}[kind]
        self._check(self.lib.pbf_set_implicit_preconditioner(self.ctx, k, int(smoothing_degree), int(coarse_degree)))
        self.bind()

    def set_newton_forcing(self, kind):
        """pbf_set_newton_forcing: 'fixed' or 'eisenstat-walker'."""
        self._check(self.lib.pbf_set_newton_forcing(self.ctx, {"fixed": 0, "eisenstat-walker": 1}[kind]))

    def implicit_step(self, T_n, rc, t, dt, cg_rtol=1e-10, cg_max_it=10000, picard_tol=1e-8,
                      picard_max_it=30, T_out=None, check=True):
        i = self.info()
        if T_out is None:
            T_out = torch.empty_like(T_n)
        it, pit, res = C.c_int(0), C.c_int(0), C.c_double(0)
        st = self.lib.pbf_implicit_step(
            self.ctx, _f64(T_n, i["n_dofs"], "T_n"), _f64(T_out, i["n_dofs"], "T_out"),
            _ptr(rc) if i["n_hist_qp"] else None, float(t), float(dt), float(cg_rtol), int(cg_max_it),
            float(picard_tol), int(picard_max_it), C.byref(it), C.byref(pit), C.byref(res),
            self._stream())
        info = dict(status=st, cg_iters=it.value, picard_iters=pit.value, rel_res=res.value)
        if check and st != 0:
            self._check(st)
        return T_out, info

    # -- dof map and octree remeshing -----------------------------------------------
    def dof_coords(self):
        x = np.zeros((self.info()["n_dofs"], 3))
        self._check(self.lib.pbf_dof_coords(self.ctx, x.ctypes.data_as(_dp)))
        return x

    def octree_info(self):
        nl, nh, ml = C.c_int64(), C.c_int64(), C.c_int()
        self._check(self.lib.pbf_octree_info(self.ctx, C.byref(nl), C.byref(nh), C.byref(ml)))
        return {"n_leaves": nl.value, "n_hanging": nh.value, "max_level": ml.value}

    def remesh(self, leaves, T, rc):
        """Move to new octree leaves; returns the transferred (T, rc).  Binds a new
        workspace (the old one is released afterwards)."""
        lv = np.ascontiguousarray(leaves, dtype=np.int32).reshape(-1, 4)
        nb, nd, nh = C.c_size_t(), C.c_int64(), C.c_int64()
        self._check(self.lib.pbf_octree_remesh_bytes(self.ctx, len(lv), lv.ctypes.data_as(C.POINTER(C.c_int32)),
                                                     C.byref(nb), C.byref(nd), C.byref(nh)))
        buf, addr = _aligned(nb.value, self.device)
        old_info = self.info()
        T_new = torch.empty(nd.value, dtype=torch.float64, device=self.device)
        rc_new = torch.empty(max(1, nh.value), dtype=torch.float64, device=self.device)
        self._check(self.lib.pbf_octree_remesh(self.ctx, C.c_void_p(addr), nb.value, _ptr(T),
                                               _ptr(rc) if old_info["n_hist_qp"] else None, _ptr(T_new),
                                               _ptr(rc_new), self._stream()))
        self.workspace = buf  # the old workspace is released here
        return T_new, rc_new

    def history_min(self, rc):
        """pbf_octree_history_min: per-leaf minima of the device history (host)."""
        out = np.ones(self.octree_info()["n_leaves"])
        self._check(self.lib.pbf_octree_history_min(self.ctx, _ptr(rc) if self.info()["n_hist_qp"] else None,
                                                    out.ctypes.data_as(_dp), self._stream()))
        return out

    def layer_leaves(self, rc_min, new_top, d_haz=4, r_coarsen=0.9):
        """pbf_octree_layer_leaves (host): leaves (n, 4) after activating the layer
        up to new_top (finest cells) on a growing octree; rc_min per leaf or None."""
        n = C.c_int64(0)
        rm = None if rc_min is None else np.ascontiguousarray(rc_min, dtype=np.float64)
        args = (self.ctx, None if rm is None else rm.ctypes.data_as(_dp), int(new_top), int(d_haz), float(r_coarsen))
        self._check(self.lib.pbf_octree_layer_leaves(*args, None, 0, C.byref(n)))
        out = np.empty((n.value, 4), dtype=np.int32)
        self._check(self.lib.pbf_octree_layer_leaves(*args, out.ctypes.data_as(C.POINTER(C.c_int32)), n.value,
                                                     C.byref(n)))
        return out

    def grow(self, leaves, new_top, T, rc):
        """Move a growing octree to new leaves with the active top new_top;
        returns the transferred (T, rc) (activated dofs at the initial
        temperature, new points as powder)."""
        lv = np.ascontiguousarray(leaves, dtype=np.int32).reshape(-1, 4)
        nb, nd, nh = C.c_size_t(), C.c_int64(), C.c_int64()
        self._check(self.lib.pbf_octree_grow_bytes(self.ctx, int(new_top), len(lv),
                                                   lv.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(nb),
                                                   C.byref(nd), C.byref(nh)))
        buf, addr = _aligned(nb.value, self.device)
        old_info = self.info()
        T_new = torch.empty(nd.value, dtype=torch.float64, device=self.device)
        rc_new = torch.empty(max(1, nh.value), dtype=torch.float64, device=self.device)
        self._check(self.lib.pbf_octree_remesh(self.ctx, C.c_void_p(addr), nb.value, _ptr(T),
                                               _ptr(rc) if old_info["n_hist_qp"] else None, _ptr(T_new),
                                               _ptr(rc_new), self._stream()))
        self.workspace = buf
        return T_new, rc_new

    # -- diagnostics ----------------------------------------------------------------
    def energy(self, T_prev, T, rc, t, dt):
        """(stored-heat change, absorbed power, Dirichlet heat flow, identity residual)."""
        i = self.info()
        out = (C.c_double * 4)()
        self._check(self.lib.pbf_energy(self.ctx, _f64(T_prev, i["n_dofs"], "T_prev"),
                                        _f64(T, i["n_dofs"], "T"), _ptr(rc) if i["n_hist_qp"] else None,
                                        float(t), float(dt), out, self._stream()))
        return tuple(out)

    def check_finite(self, x):
        """(all finite, max |x| over the finite values)."""
        ok, mx = C.c_int(0), C.c_double(0)
        st = self.lib.pbf_check_finite(self.ctx, _ptr(x), x.numel(), C.byref(ok), C.byref(mx),
                                       self._stream())
        if st not in (0, -6):
            self._check(st)
        return bool(ok.value), mx.value

    # -- probes and adjoint -------------------------------------------------------
    def set_probes(self, pts, targets=None):
        p = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
        t = None if targets is None else np.ascontiguousarray(targets, dtype=np.float64)
        if t is not None and t.size != len(p):
            raise ValueError("one target per probe")
        self._check(self.lib.pbf_set_probes(self.ctx, len(p), p.ctypes.data_as(_dp),
                                            None if t is None else t.ctypes.data_as(_dp),
                                            self._stream()))
        self.n_probes = len(p)

    def probe(self, T):
        i = self.info()
        vals = torch.empty(max(1, self.n_probes), dtype=torch.float64, device=self.device)
        self._check(self.lib.pbf_probe(self.ctx, _f64(T, i["n_dofs"], "T"), _ptr(vals), self._stream()))
        return vals[: self.n_probes]

    def objective(self, T):
        """(J as a one-element device tensor, dJ/dT)."""
        i = self.info()
        J = torch.empty(1, dtype=torch.float64, device=self.device)
        lam = torch.empty_like(T)
        self._check(self.lib.pbf_objective(self.ctx, _f64(T, i["n_dofs"], "T"), _ptr(J), _ptr(lam),
                                           self._stream()))
        return J, lam

    def adjoint_step(self, T_n, T_next, rc_prev, lam_next, mu, t_n, dt, dJdW, lam=None):
        i = self.info()
        if lam is None:
            lam = torch.empty_like(lam_next)
        h = i["n_hist_qp"] > 0
        self._check(self.lib.pbf_adjoint_step(
            self.ctx, _f64(T_n, i["n_dofs"], "T_n"), _f64(T_next, i["n_dofs"], "T_next"), _ptr(rc_prev) if h else None,
            _f64(lam_next, i["n_dofs"], "lam_next"), _f64(lam, i["n_dofs"], "lam"),
            _ptr(mu) if h else None, float(t_n), float(dt), _ptr(dJdW) if self.n_tracks else None,
            self._stream()))
        return lam

    def gradient_work(self, n_snaps):
        """Device buffer for gradient_forward/backward with n_snaps slots."""
        nb = C.c_size_t()
        self._check(self.lib.pbf_adjoint_work_bytes(self.ctx, int(n_snaps), C.byref(nb)))
        buf, addr = _aligned(nb.value, self.device)
        return {"buf": buf, "addr": addr, "bytes": nb.value, "n_snaps": int(n_snaps)}

    def gradient_forward(self, T0, rc0, t0, dt, n_steps, work):
        i = self.info()
        T_N = torch.empty(i["n_dofs"], dtype=torch.float64, device=self.device)
        J = torch.empty(1, dtype=torch.float64, device=self.device)
        self._check(self.lib.pbf_gradient_forward(
            self.ctx, _f64(T0, i["n_dofs"], "T0"), _ptr(rc0) if i["n_hist_qp"] else None, float(t0),
            float(dt), int(n_steps), work["n_snaps"], C.c_void_p(work["addr"]), work["bytes"],
            _ptr(T_N), _ptr(J), self._stream()))
        return T_N, J

    def gradient_backward(self, t0, dt, n_steps, work, with_lam0=False):
        i = self.info()
        K = max(1, self.n_tracks)
        out = {k: torch.zeros(K, dtype=torch.float64, device=self.device) for k in ("dJdW", "dJdP")}
        out["dJdA"] = torch.zeros(1, dtype=torch.float64, device=self.device)
        out["lam0"] = torch.empty(i["n_dofs"], dtype=torch.float64, device=self.device) if with_lam0 else None
        adv = C.c_int64(0)
        self._check(self.lib.pbf_gradient_backward(
            self.ctx, float(t0), float(dt), int(n_steps), work["n_snaps"], C.c_void_p(work["addr"]),
            work["bytes"], _ptr(out["dJdW"]), _ptr(out["dJdP"]), _ptr(out["dJdA"]), _ptr(out["lam0"]),
            C.byref(adv), self._stream()))
        out["dJdW"] = out["dJdW"][: self.n_tracks]
        out["dJdP"] = out["dJdP"][: self.n_tracks]
        out["n_advances"] = adv.value
        return out

    def timing_begin(self, max_steps, every=1):
        """Record kernel events on every `every`-th explicit step (at most max_steps)."""
        self._check(self.lib.pbf_timing_begin(self.ctx, int(max_steps), int(every)))

    def timing_end(self):
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        self._check(self.lib.pbf_timing_end(self.ctx, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value


def from_problem(prob, device="cuda:0", leaves=None, active_layers=None, bind=True, top=None):
    """Simulation set up from a problem description object with the attributes
    of pbf_workloads.Problem (argument marshalling only); an octree mesh when the
    problem (or the `leaves` argument) holds leaves; a growing box with the bottom
    active_layers cell layers active when given; no workspace is bound when
    bind is False."""
    lv = leaves if leaves is not None else getattr(prob, "leaves", None)
    s = Simulation(prob.degree, prob.nx, prob.ny, prob.nz, prob.L, device=device,
                   max_level=getattr(prob, "max_level", 0), leaves=lv, top=top)
    s.set_dirichlet(prob.dirichlet_mask, prob.T_D)
    s.set_material(prob.T_bp, prob.k_bp, prob.cp_bp, prob.rho, prob.T_s, prob.T_l, prob.latent,
                   prob.powder_k_factor, prob.powder_depth)
    s.set_laser(prob.laser_kind, prob.radius, prob.absorptivity, prob.h_powder, prob.t_start,
                prob.tracks)
    if getattr(prob, "emissivity", 0.0) or getattr(prob, "evap_on", False):
        t_inf = getattr(prob, "T_inf", None)
        s.set_surface_loss(prob.emissivity, prob.T_D if t_inf is None else t_inf, prob.evap_on, prob.T_v,
                           prob.C_P, prob.C_T, prob.C_M, prob.h_v, prob.T_h0, prob.dT_max)
    if active_layers is not None:
        s.set_active_layers(active_layers)
    if bind:
        s.bind()
    return s
