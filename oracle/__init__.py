"""ctypes wrapper of the plain C oracle (oracle.c on boxes, octree.c on octrees).

TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.  See oracle.h for the
definitions each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)


class OrProblem(C.Structure):
    _fields_ = [
        ("degree", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("Lx", C.c_double), ("Ly", C.c_double), ("Lz", C.c_double),
        ("dirichlet_mask", C.c_uint), ("T_D", C.c_double),
        ("n_bp", C.c_int), ("T_bp", _dp), ("k_bp", _dp), ("cp_bp", _dp),
        ("rho", C.c_double), ("T_s", C.c_double), ("T_l", C.c_double), ("latent", C.c_double),
        ("powder_k_factor", C.c_double), ("powder_depth", C.c_double),
        ("laser_kind", C.c_int), ("radius", C.c_double), ("absorptivity", C.c_double),
        ("h_powder", C.c_double), ("t_start", C.c_double),
        ("n_tracks", C.c_int), ("tracks", _dp), ("track_power", _dp),
        ("emissivity", C.c_double), ("T_inf", C.c_double), ("evap_on", C.c_int),
        ("T_v", C.c_double), ("C_P", C.c_double), ("C_T", C.c_double), ("C_M", C.c_double),
        ("h_v", C.c_double), ("T_h0", C.c_double), ("dT_max", C.c_double),
    ]


_SOURCES = ("oracle.c", "octree.c")
_HEADERS = ("oracle.h", "oracle_internal.h")


def build(force: bool = False) -> str:
    srcs = [os.path.join(_HERE, f) for f in _SOURCES]
    newest = max(os.path.getmtime(os.path.join(_HERE, f)) for f in _SOURCES + _HEADERS)
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < newest:
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-o", _SO,
                               *srcs, "-lm"])
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        P = C.POINTER(OrProblem)
        L.or_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
        L.or_lagrange.argtypes = [C.c_int, C.c_int, C.c_double]
        L.or_lagrange.restype = C.c_double
        L.or_lagrange_deriv.argtypes = [C.c_int, C.c_int, C.c_double]
        L.or_lagrange_deriv.restype = C.c_double
        for nm in ("or_liquid_fraction", "or_capacity"):
            getattr(L, nm).argtypes = [P, C.c_double]
            getattr(L, nm).restype = C.c_double
        L.or_conductivity.argtypes = [P, C.c_double, C.c_double]
        L.or_conductivity.restype = C.c_double
        L.or_beam.argtypes = [P, C.c_double, _dp, _dp, _dp, C.POINTER(C.c_int)]
        L.or_volume_source.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double]
        L.or_volume_source.restype = C.c_double
        L.or_surface_source.argtypes = [P, C.c_double, C.c_double, C.c_double]
        L.or_surface_source.restype = C.c_double
        L.or_surface_loss.argtypes = [P, C.c_double]
        L.or_surface_loss.restype = C.c_double
        L.or_surface_loss_vector.argtypes = [P, _dp, _dp]
        L.or_jacobian_apply.argtypes = [P, _dp, _dp, _dp, C.c_double, _dp, _dp]
        L.or_activate_layers.argtypes = [P, C.c_int, C.c_int, C.c_double, _dp, _dp]
        L.or_picard_apply.argtypes = [P, _dp, _dp, _dp, C.c_double, _dp, _dp]
        L.or_implicit_residual.argtypes = [P, _dp, _dp, _dp, C.c_double, C.c_double, _dp]
        L.or_implicit_step_newton.argtypes = [P, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                              C.c_double, C.c_int, _dp, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                              C.POINTER(C.c_double)]
        L.or_n_dofs.argtypes = [P]
        L.or_n_dofs.restype = C.c_int64
        L.or_n_qp.argtypes = [P]
        L.or_n_qp.restype = C.c_int64
        L.or_init_history.argtypes = [P, _dp]
        L.or_assemble.argtypes = [P, _dp, _dp, C.c_double, _dp, _dp, _dp]
        L.or_assemble_lagged.argtypes = [P, _dp, _dp, C.c_double, _dp, _dp, _dp]
        L.or_explicit_steps.argtypes = [P, _dp, _dp, C.c_double, C.c_double, C.c_int]
        L.or_explicit_step_sampled.argtypes = [P, _dp, _dp, C.c_double, C.c_double, C.c_int, _i64p,
                                               _dp]
        L.or_stability_lambda.argtypes = [P, _dp, C.c_int]
        L.or_stability_lambda.restype = C.c_double
        L.or_capacity_apply.argtypes = [P, _dp, _dp, _dp]
        L.or_implicit_step.argtypes = [P, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int,
                                       C.c_double, C.c_int, _dp, C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), _dp]
        L.or_probe.argtypes = [P, _dp, C.c_int, _dp, _dp]
        L.or_adjoint_run.argtypes = [P, _dp, C.c_double, C.c_double, C.c_int, C.c_int, _dp, _dp,
                                     _dp, _dp, _dp, _dp]
        O = C.c_void_p
        L.or_oct_build.argtypes = [P, C.c_int, C.c_int64, _i64p]
        L.or_oct_build.restype = O
        L.or_oct_build_top.argtypes = [P, C.c_int, C.c_int64, _i64p, C.c_int64]
        L.or_oct_build_top.restype = O
        L.or_oct_free.argtypes = [O]
        L.or_oct_free.restype = None
        for nm in ("or_oct_n_dofs", "or_oct_n_hanging", "or_oct_n_qp"):
            getattr(L, nm).argtypes = [O]
            getattr(L, nm).restype = C.c_int64
        L.or_oct_dof_coords.argtypes = [O, _dp]
        L.or_oct_dof_coords.restype = None
        L.or_oct_dirichlet.argtypes = [O, C.POINTER(C.c_int)]
        L.or_oct_dirichlet.restype = None
        L.or_oct_init_history.argtypes = [O, _dp]
        L.or_oct_init_history.restype = None
        L.or_oct_assemble.argtypes = [O, _dp, _dp, C.c_double, _dp, _dp, _dp, C.c_int]
        L.or_oct_explicit_steps.argtypes = [O, _dp, _dp, C.c_double, C.c_double, C.c_int]
        L.or_oct_stability_lambda.argtypes = [O, _dp, C.c_int]
        L.or_oct_stability_lambda.restype = C.c_double
        L.or_oct_implicit_step.argtypes = [O, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int,
                                           C.c_double, C.c_int, _dp, C.POINTER(C.c_int),
                                           C.POINTER(C.c_int), _dp]
        L.or_oct_probe.argtypes = [O, _dp, C.c_int, _dp, _dp]
        L.or_oct_transfer.argtypes = [O, _dp, _dp, O, _dp, _dp]
        L.or_oct_transfer_growing.argtypes = [O, _dp, _dp, O, C.c_double, _dp, _dp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


class Oracle:
    """Holds one problem description (a pbf_workloads.Problem or anything with the
    same attributes) and exposes the oracle's functions on numpy arrays."""

    def __init__(self, prob, track_power=None):
        self.prob = prob
        self._keep = []

        def arr(x):
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
            self._keep.append(a)
            return a

        tb, kb, cb = arr(prob.T_bp), arr(prob.k_bp), arr(prob.cp_bp)
        tr = arr(np.asarray(prob.tracks, dtype=np.float64).reshape(-1, 8))
        s = OrProblem()
        s.degree, s.nx, s.ny, s.nz = prob.degree, prob.nx, prob.ny, prob.nz
        s.Lx, s.Ly, s.Lz = prob.L
        s.dirichlet_mask = prob.dirichlet_mask
        s.T_D = prob.T_D
        s.n_bp = len(tb)
        s.T_bp, s.k_bp, s.cp_bp = _ptr(tb), _ptr(kb), _ptr(cb)
        s.rho, s.T_s, s.T_l, s.latent = prob.rho, prob.T_s, prob.T_l, prob.latent
        s.powder_k_factor, s.powder_depth = prob.powder_k_factor, prob.powder_depth
        s.laser_kind, s.radius, s.absorptivity = prob.laser_kind, prob.radius, prob.absorptivity
        s.h_powder, s.t_start = prob.h_powder, prob.t_start
        s.n_tracks = tr.shape[0]
        s.tracks = _ptr(tr) if tr.size else None
        if track_power is not None:
            s.track_power = _ptr(arr(track_power))
        else:
            s.track_power = None
        s.emissivity = getattr(prob, "emissivity", 0.0)
        t_inf = getattr(prob, "T_inf", None)
        s.T_inf = prob.T_D if t_inf is None else t_inf
        s.evap_on = 1 if getattr(prob, "evap_on", False) else 0
        for name, default in (("T_v", 3000.0), ("C_P", 54.0e3), ("C_T", 5.0e4), ("C_M", 1.0e-3),
                              ("h_v", 6.0e6), ("T_h0", 663.0), ("dT_max", 1000.0)):
            setattr(s, name, getattr(prob, name, default))
        self.s = s
        self.L = lib()
        self.N = int(self.L.or_n_dofs(C.byref(s)))
        self.NQ = int(self.L.or_n_qp(C.byref(s)))

    # -- state ---------------------------------------------------------------
    def init_T(self) -> np.ndarray:
        T = np.full(self.N, float(self.prob.T0))
        m = self.dirichlet_mask()
        T[m] = self.prob.T_D
        return T

    def init_history(self) -> np.ndarray:
        rc = np.zeros(self.NQ)
        self.L.or_init_history(C.byref(self.s), _ptr(rc))
        return rc

    def dirichlet_mask(self) -> np.ndarray:
        p = self.prob
        NX, NY, NZ = p.nodes_per_dim
        k, j, i = np.meshgrid(np.arange(NZ), np.arange(NY), np.arange(NX), indexing="ij")
        m = p.dirichlet_mask
        d = np.zeros((NZ, NY, NX), dtype=bool)
        if m & 1: d |= i == 0
        if m & 2: d |= i == NX - 1
        if m & 4: d |= j == 0
        if m & 8: d |= j == NY - 1
        if m & 16: d |= k == 0
        if m & 32: d |= k == NZ - 1
        return d.reshape(-1)

    # -- explicit scheme -----------------------------------------------------------
    def assemble(self, T, rc, t):
        T = np.ascontiguousarray(T, dtype=np.float64)
        f, Cl, fv = np.zeros(self.N), np.zeros(self.N), np.zeros(self.N)
        self.L.or_assemble(C.byref(self.s), _ptr(T), _ptr(rc), t, _ptr(f), _ptr(Cl), _ptr(fv))
        return f, Cl, fv

    def assemble_lagged(self, T, rc, t):
        T = np.ascontiguousarray(T, dtype=np.float64)
        f, Cl, fv = np.zeros(self.N), np.zeros(self.N), np.zeros(self.N)
        self.L.or_assemble_lagged(C.byref(self.s), _ptr(T), _ptr(rc), t, _ptr(f), _ptr(Cl), _ptr(fv))
        return f, Cl, fv

    def explicit_steps(self, T, rc, t0, dt, n):
        self.L.or_explicit_steps(C.byref(self.s), _ptr(T), _ptr(rc), t0, dt, n)
        return T

    def activate_layers(self, nz_old, nz_new, T0, T, rc):
        """On the whole box: layers nz_old..nz_new-1 become active (T0, new powder), in place."""
        self.L.or_activate_layers(C.byref(self.s), int(nz_old), int(nz_new), float(T0), _ptr(T), _ptr(rc))

    def surface_loss_vector(self, T):
        """f_RE(T): the radiation and evaporation terms alone, assembled."""
        T = np.ascontiguousarray(T, dtype=np.float64)
        f = np.zeros(self.N)
        self.L.or_surface_loss_vector(C.byref(self.s), _ptr(T), _ptr(f))
        return f

    def explicit_step_sampled(self, T, rc, t, dt, nodes):
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        out = np.zeros(len(nodes))
        self.L.or_explicit_step_sampled(C.byref(self.s), _ptr(T), _ptr(rc), t, dt, len(nodes),
                                        nodes.ctypes.data_as(_i64p), _ptr(out))
        return out

    def stability_lambda(self, v0, iters):
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        return float(self.L.or_stability_lambda(C.byref(self.s), _ptr(v0), iters))

    # -- implicit scheme -------------------------------------------------------------
    def capacity_apply(self, Tn, x):
        y = np.zeros(self.N)
        self.L.or_capacity_apply(C.byref(self.s), _ptr(np.ascontiguousarray(Tn)),
                                 _ptr(np.ascontiguousarray(x)), _ptr(y))
        return y

    def implicit_step(self, Tn, rc, t, dt, cg_rtol=1e-10, cg_max_it=10000, picard_tol=1e-8,
                      picard_max_it=30):
        out = np.zeros(self.N)
        it, pit, res = C.c_int(0), C.c_int(0), C.c_double(0)
        st = self.L.or_implicit_step(C.byref(self.s), _ptr(np.ascontiguousarray(Tn)), _ptr(rc), t, dt,
                                     cg_rtol, cg_max_it, picard_tol, picard_max_it, _ptr(out),
                                     C.byref(it), C.byref(pit), C.byref(res))
        return out, dict(status=st, cg_iters=it.value, picard_iters=pit.value, rel_res=res.value)

    def picard_apply(self, Tn, Ti, rc, dt, x):
        """y = (C(T_n)/dt + K(T^i)) x, the symmetric part of the Jacobian."""
        y = np.zeros(self.N)
        c = np.ascontiguousarray
        self.L.or_picard_apply(C.byref(self.s), _ptr(c(Tn)), _ptr(c(Ti)), _ptr(c(rc)), dt, _ptr(c(x)), _ptr(y))
        return y

    def jacobian_apply(self, Tn, Ti, rc, dt, x):
        """y = J(T^i) x of the implicit residual (Newton, eq. Newton_1)."""
        y = np.zeros(self.N)
        c = np.ascontiguousarray
        self.L.or_jacobian_apply(C.byref(self.s), _ptr(c(Tn)), _ptr(c(Ti)), _ptr(c(rc)), dt, _ptr(c(x)), _ptr(y))
        return y

    def implicit_residual(self, Tn, T, rc, t, dt):
        r = np.zeros(self.N)
        c = np.ascontiguousarray
        self.L.or_implicit_residual(C.byref(self.s), _ptr(c(Tn)), _ptr(c(T)), _ptr(c(rc)), t, dt, _ptr(r))
        return r

    def implicit_step_newton(self, Tn, rc, t, dt, lin_rtol=1e-10, restart=30, lin_max_it=5000,
                             newton_tol=1e-8, newton_max_it=30):
        out = np.zeros(self.N)
        it, nit, res = C.c_int(0), C.c_int(0), C.c_double(0)
        st = self.L.or_implicit_step_newton(C.byref(self.s), _ptr(np.ascontiguousarray(Tn)), _ptr(rc), t, dt,
                                            lin_rtol, restart, lin_max_it, newton_tol, newton_max_it, _ptr(out),
                                            C.byref(it), C.byref(nit), C.byref(res))
        return out, dict(status=st, lin_iters=it.value, newton_iters=nit.value, rel_res=res.value)

    # -- probes and adjoint ---------------------------------------------------------
    def probe(self, T, pts):
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        vals = np.zeros(len(pts))
        self.L.or_probe(C.byref(self.s), _ptr(np.ascontiguousarray(T)), len(pts), _ptr(pts), _ptr(vals))
        return vals

    def adjoint(self, T0, t0, dt, n_steps, pts, targets, with_lam0=False):
        """J, dJ/dW_eff per track and T_N (and dJ/dT_0 if with_lam0) of n_steps
        explicit steps from T0 and the initial history."""
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        tg = np.ascontiguousarray(targets, dtype=np.float64)
        J = C.c_double(0)
        dW = np.zeros(max(1, self.s.n_tracks))
        TN = np.zeros(self.N)
        lam0 = np.zeros(self.N) if with_lam0 else None
        rc = self.L.or_adjoint_run(C.byref(self.s), _ptr(np.ascontiguousarray(T0)), t0, dt, n_steps,
                                   len(pts), _ptr(pts), _ptr(tg), C.byref(J), _ptr(dW), _ptr(TN),
                                   _ptr(lam0) if with_lam0 else None)
        if rc == -2:
            raise ValueError("the oracle adjoint covers the model without surface losses")
        if with_lam0:
            return J.value, dW[: self.s.n_tracks], TN, lam0
        return J.value, dW[: self.s.n_tracks], TN

    # -- scalar material law and laser (for pins) ------------------------------------
    def surface_loss(self, T):
        """Outward heat flux density q_rad + q_evap through the free surface at T."""
        return self.L.or_surface_loss(C.byref(self.s), T)

    def liquid_fraction(self, T):
        return self.L.or_liquid_fraction(C.byref(self.s), T)

    def conductivity(self, T, rc):
        return self.L.or_conductivity(C.byref(self.s), T, rc)

    def capacity(self, T):
        return self.L.or_capacity(C.byref(self.s), T)

    def beam(self, t):
        xb, yb, W, k = C.c_double(), C.c_double(), C.c_double(), C.c_int(-1)
        on = self.L.or_beam(C.byref(self.s), t, C.byref(xb), C.byref(yb), C.byref(W), C.byref(k))
        return bool(on), xb.value, yb.value, W.value, k.value


class OctOracle:
    """The oracle on an octree mesh: prob is a problem description with coarse
    cells nx, ny, nz, max_level and leaves (n, 4) = (level, ix, iy, iz)."""

    def __init__(self, prob, leaves=None, track_power=None, top=None):
        """top (finest cells): the active top of a growing build (leaves cover
        z < top); None: the box top."""
        self.base = Oracle(prob, track_power=track_power)  # holds the problem struct
        self.L = self.base.L
        lv = np.ascontiguousarray(prob.leaves if leaves is None else leaves, dtype=np.int64)
        self._leaves = lv
        if top is None:
            self.h = self.L.or_oct_build(C.byref(self.base.s), int(prob.max_level), len(lv),
                                         lv.ctypes.data_as(_i64p))
        else:
            self.h = self.L.or_oct_build_top(C.byref(self.base.s), int(prob.max_level), len(lv),
                                             lv.ctypes.data_as(_i64p), int(top))
        if not self.h:
            raise RuntimeError("or_oct_build failed")
        self.prob = prob
        self.N = self.L.or_oct_n_dofs(self.h)
        self.NQ = self.L.or_oct_n_qp(self.h)
        self.n_hanging = self.L.or_oct_n_hanging(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            self.L.or_oct_free(self.h)
            self.h = None

    def dof_coords(self):
        x = np.zeros((self.N, 3))
        self.L.or_oct_dof_coords(self.h, _ptr(x))
        return x

    def dirichlet_mask(self):
        f = np.zeros(self.N, dtype=np.int32)
        self.L.or_oct_dirichlet(self.h, f.ctypes.data_as(C.POINTER(C.c_int)))
        return f.astype(bool)

    def init_T(self):
        T = np.full(self.N, float(self.prob.T0))
        T[self.dirichlet_mask()] = self.prob.T_D
        return T

    def init_history(self):
        rc = np.zeros(self.NQ)
        self.L.or_oct_init_history(self.h, _ptr(rc))
        return rc

    def assemble(self, T, rc, t, hist=0):
        T = np.ascontiguousarray(T, dtype=np.float64)
        f, Cl, fv = np.zeros(self.N), np.zeros(self.N), np.zeros(self.N)
        self.L.or_oct_assemble(self.h, _ptr(T), _ptr(rc), t, _ptr(f), _ptr(Cl), _ptr(fv), hist)
        return f, Cl, fv

    def explicit_steps(self, T, rc, t0, dt, n):
        self.L.or_oct_explicit_steps(self.h, _ptr(T), _ptr(rc), t0, dt, n)
        return T

    def stability_lambda(self, v0, iters):
        return self.L.or_oct_stability_lambda(self.h, _ptr(np.ascontiguousarray(v0, dtype=np.float64)), iters)

    def implicit_step(self, Tn, rc, t, dt, cg_rtol=1e-10, cg_max_it=10000, picard_tol=1e-8,
                      picard_max_it=30):
        out = np.zeros(self.N)
        it, pit, res = C.c_int(0), C.c_int(0), C.c_double(0)
        st = self.L.or_oct_implicit_step(self.h, _ptr(np.ascontiguousarray(Tn)), _ptr(rc), t, dt, cg_rtol,
                                         cg_max_it, picard_tol, picard_max_it, _ptr(out), C.byref(it),
                                         C.byref(pit), C.byref(res))
        return out, dict(status=st, cg_iters=it.value, picard_iters=pit.value, rel_res=res.value)

    def probe(self, T, pts):
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        vals = np.zeros(len(pts))
        if self.L.or_oct_probe(self.h, _ptr(np.ascontiguousarray(T)), len(pts), _ptr(pts), _ptr(vals)):
            raise ValueError("probe outside the mesh")
        return vals

    def transfer_growing(self, T, rc, new, T0):
        """(T, history) across the adaptation and layer activation of a growing
        build, onto the octree `new` (an OctOracle with a higher or equal top)."""
        Tn, rn = np.zeros(new.N), np.zeros(new.NQ)
        if self.L.or_oct_transfer_growing(self.h, _ptr(np.ascontiguousarray(T)), _ptr(rc), new.h, float(T0),
                                          _ptr(Tn), _ptr(rn)):
            raise ValueError("transfer: a new point lies outside the old mesh")
        return Tn, rn

    def transfer(self, T, rc, new):
        """(T, history) on the octree `new` (an OctOracle) from this one."""
        Tn, rn = np.zeros(new.N), np.zeros(new.NQ)
        if self.L.or_oct_transfer(self.h, _ptr(np.ascontiguousarray(T)), _ptr(rc), new.h, _ptr(Tn), _ptr(rn)):
            raise ValueError("transfer: a new point lies outside the old mesh")
        return Tn, rn


def gauss_legendre(n):
    x, w = np.zeros(n), np.zeros(n)
    lib().or_gauss_legendre(n, _ptr(x), _ptr(w))
    return x, w


def lagrange(p, a, x):
    return lib().or_lagrange(p, a, x)


def lagrange_deriv(p, a, x):
    return lib().or_lagrange_deriv(p, a, x)
