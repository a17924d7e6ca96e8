"""Thin ctypes binding of libwq.so (C ABI declared in include/wq.h).

Argument marshalling only: every step of the weighted-quadrature path runs in the HIP
kernels of libwq.so. PyTorch supplies device memory (tensors) and streams. The library
must have been built (paper_2605_29334_amd/build.py); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwq.so")

WQ_FAM_MASS, WQ_FAM_DX, WQ_FAM_DY, WQ_FAM_LAP, WQ_FAM_DZ = 1, 2, 4, 8, 16
WQ_FP64, WQ_SPLIT_FP16, WQ_SPLIT_BF16, WQ_SLICED_FP16 = 0, 1, 2, 3
ARR_ROW_PTR, ARR_COL, ARR_QPTR, ARR_QIDX, ARR_ETYPE, ARR_S, ARR_X, ARR_DETJ = range(8)
_ARR_DTYPE = {ARR_ROW_PTR: torch.int64, ARR_COL: torch.int32, ARR_QPTR: torch.int64, ARR_QIDX: torch.int32,
              ARR_ETYPE: torch.uint8, ARR_S: torch.uint8, ARR_X: torch.float64, ARR_DETJ: torch.float64}


class WQError(RuntimeError):
    def __init__(self, status, where):
        lib = _lib()
        super().__init__(f"{where}: {lib.wq_strerror(status).decode()} ({status}): {lib.wq_last_error().decode()}")
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nf", C.c_int32), ("n_fn", C.c_int32),
                ("face_vtx", C.c_void_p), ("split", C.c_void_p), ("ext_ptr", C.c_void_p),
                ("ext_fn", C.c_void_p), ("coef_ptr", C.c_void_p), ("coef", C.c_void_p), ("ctrl", C.c_void_p),
                ("dim", C.c_int32)]


class Timing(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("ms", C.c_double), ("work", C.c_int64)]


class SolveReport(C.Structure):
    _fields_ = [("systems", C.c_int64), ("truncated", C.c_int64), ("max_sweeps", C.c_int32),
                ("min_kept_ratio", C.c_double), ("max_dropped_ratio", C.c_double), ("certified", C.c_int64)]


class Conductivity(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a", C.c_double), ("b", C.c_double)]


TANGENT_SYMMETRIC, TANGENT_EXACT = 0, 1


class HeatParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("theta", C.c_double), ("k", Conductivity), ("tol", C.c_double),
                ("max_newton", C.c_int32), ("cg_rtol", C.c_double), ("max_cg", C.c_int32), ("tangent", C.c_int32)]


class HeatReport(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("cg_iters", C.c_int32), ("residual0", C.c_double),
                ("residual", C.c_double)]


K_LINEAR, K_QUADRATIC, K_EXP, K_SIN = 0, 1, 2, 3
SOURCE_NONE, SOURCE_MANUFACTURED = 0, 1


class Request(C.Structure):
    _fields_ = [("mesh", MeshDesc), ("dirichlet", C.c_void_p), ("heat", HeatParams), ("n_steps", C.c_int32),
                ("source", C.c_int32), ("lam", C.c_double), ("reuse_setup", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_iters", C.c_int32), ("cg_iters", C.c_int32), ("n_rows", C.c_int64),
                ("nnz", C.c_int64), ("residual", C.c_double), ("submitted", C.c_double), ("started", C.c_double),
                ("finished", C.c_double), ("hbm_estimate", C.c_size_t), ("setup_reused", C.c_int32),
                ("joined", C.c_int32)]

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2605_29334_amd/build.py")
        lib = C.CDLL(LIB_PATH)
        P, I64, I32, U, D = C.c_void_p, C.c_int64, C.c_int32, C.c_uint, C.c_double
        sig = {
            "wq_mesh_create": ([P, P], C.c_int),
            "wq_mesh_destroy": ([P], None),
            "build_points": ([P, C.c_int, P, P, P, P, P], C.c_int),
            "build_points_with_s": ([P, P, C.c_int, P, P, P, P, P], C.c_int),
            "wq_points_destroy": ([P], None),
            "wq_points_size": ([P, C.c_int], I64),
            "wq_points_get": ([P, C.c_int, P, P], C.c_int),
            "wq_points_info": ([P, C.c_int], I64),
            "solve_weights": ([P, P, U, D, P, P, P], C.c_int),
            "wq_weights_destroy": ([P], None),
            "wq_weights_get": ([P, C.c_int, P, P], C.c_int),
            "wq_rhs_get": ([P, C.c_int, P, P], C.c_int),
            "assemble_mass": ([P, P, P, P, C.c_int, P], C.c_int),
            "assemble_stiffness": ([P, P, P, P, C.c_int, P], C.c_int),
            "assemble_biharmonic": ([P, P, P, P, C.c_int, P], C.c_int),
            "assemble_mass_stiffness": ([P, P, P, P, P, P, C.c_int, P], C.c_int),
            "assemble_tangent": ([P, P, P, P, D, Conductivity, P, P, P, C.c_int, P], C.c_int),
            "assemble_tangent_noalloc": ([P, P, P, P, D, Conductivity, P, P, P, C.c_int, P], C.c_int),
            "assemble_tangent_exact": ([P, P, P, P, D, Conductivity, P, P, P, C.c_int, P], C.c_int),
            "wq_heat_step": ([P, P, C.POINTER(HeatParams), P, P, P, P, P, P, C.POINTER(HeatReport), P], C.c_int),
            "wq_server_start": ([C.c_size_t, C.c_int32, P], C.c_int),
            "wq_server_submit": ([P, C.POINTER(Request), P, P], C.c_int),
            "wq_server_poll": ([P, C.c_int64, C.c_int, C.POINTER(Result)], C.c_int),
            "wq_server_stop": ([P], None),
            "wq_server_set_join": ([P, C.c_int32, C.c_int64], C.c_int),
            "wq_set_side_streams": ([C.c_int32], C.c_int),
            "wq_batch_create": ([P, C.c_int32, P], C.c_int),
            "wq_batch_build": ([P, U, D, P, P], C.c_int),
            "wq_batch_info": ([P, C.c_int32, P, P, P, P, P, P], C.c_int),
            "wq_batch_points": ([P], P),
            "wq_batch_weights": ([P], P),
            "wq_batch_graph_assemble": ([P, P, P, P, P, C.c_int, P], C.c_int),
            "wq_batch_destroy": ([P], None),
            "wq_autotune_assembly": ([P, P, P, P, P], C.c_int),
            "wq_autotune_tiles": ([P, P, P, P, P, P], C.c_int),
            "gauss_setup": ([P, P, C.c_int, P, P], C.c_int),
            "wq_gauss_destroy": ([P], None),
            "wq_gauss_size": ([P], I64),
            "wq_gauss_get_x": ([P, P, P], C.c_int),
            "assemble_gauss": ([P, C.c_int, P, P, P], C.c_int),
            "wq_timing_enable": ([C.c_int], None),
            "wq_timings": ([P, C.c_int], C.c_int),
            "wq_strerror": ([C.c_int], C.c_char_p),
            "wq_last_error": ([], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        del I32
        _LIB = lib
    return _LIB


def exported_symbols():
    """Names the C ABI declares (checked by the CPU tests against the built library)."""
    return ["wq_mesh_create", "wq_mesh_destroy", "build_points", "build_points_with_s", "wq_points_destroy",
            "wq_points_size", "wq_points_info", "wq_points_get", "solve_weights", "wq_weights_destroy", "wq_weights_get",
            "wq_rhs_get", "assemble_mass", "assemble_stiffness", "assemble_biharmonic", "assemble_mass_stiffness",
            "assemble_tangent", "assemble_tangent_noalloc", "assemble_tangent_exact", "wq_heat_step", "wq_server_start", "wq_server_submit", "wq_server_poll",
            "wq_server_stop", "wq_server_set_join", "wq_batch_create", "wq_batch_build", "wq_batch_info", "wq_batch_points",
            "wq_batch_weights", "wq_batch_graph_assemble", "wq_batch_destroy", "wq_autotune_assembly", "wq_autotune_tiles",
            "gauss_setup", "wq_gauss_destroy", "wq_gauss_size", "wq_gauss_get_x", "assemble_gauss",
            "wq_timing_enable", "wq_timings", "wq_set_side_streams", "wq_strerror", "wq_last_error"]


def _check(status, where):
    if status != 0:
        raise WQError(status, where)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Mesh:
    """wq_mesh_create on a fixture dict (host arrays are copied to the current device)."""

    def __init__(self, fx):
        self._keep = {
            "face_vtx": np.ascontiguousarray(fx["face_vtx"], dtype=np.int32),
            "split": np.ascontiguousarray(fx["split"], dtype=np.uint8),
            "ext_ptr": np.ascontiguousarray(fx["ext_ptr"], dtype=np.int64),
            "ext_fn": np.ascontiguousarray(fx["ext_fn"], dtype=np.int32),
            "coef_ptr": np.ascontiguousarray(fx["coef_ptr"], dtype=np.int64),
            "coef": np.ascontiguousarray(fx["coef"], dtype=np.float64),
            "ctrl": np.ascontiguousarray(fx["ctrl"], dtype=np.float64),
        }
        k = self._keep
        d = MeshDesc(int(fx["nv"]), int(len(k["face_vtx"])), int(fx["n_fn"]),
                     *[C.c_void_p(k[n].ctypes.data) for n in ("face_vtx", "split", "ext_ptr", "ext_fn",
                                                              "coef_ptr", "coef", "ctrl")], int(k["ctrl"].shape[1]))
        h = C.c_void_p()
        _check(_lib().wq_mesh_create(C.byref(d), C.byref(h)), "wq_mesh_create")
        self.h = h
        self.nf = len(k["face_vtx"])
        self.n_fn = int(fx["n_fn"])
        self.dim = int(k["ctrl"].shape[1])

    def close(self):
        if self.h:
            _lib().wq_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Points:
    """build_points: classification, points, pattern, point sets, basis at points."""

    def __init__(self, mesh, want_laplacian=False, stream=None, s_init=None):
        h = C.c_void_p()
        n, nnz, npt = C.c_int64(), C.c_int64(), C.c_int64()
        if s_init is None:
            st = _lib().build_points(mesh.h, int(want_laplacian), _stream(stream), C.byref(h), C.byref(n),
                                     C.byref(nnz), C.byref(npt))
        else:
            s_arr = np.ascontiguousarray(s_init, dtype=np.uint8)
            st = _lib().build_points_with_s(mesh.h, C.c_void_p(s_arr.ctypes.data), int(want_laplacian),
                                            _stream(stream), C.byref(h), C.byref(n), C.byref(nnz), C.byref(npt))
        _check(st, "build_points")
        self.h = h
        self.mesh = mesh
        self.n_rows, self.nnz, self.n_points = n.value, nnz.value, npt.value

    def info(self):
        keys = ["max_row", "max_r", "cells", "tiles", "tile_entries", "max_tile_nnz", "max_tile_entries",
                "max_tile_members", "pairs", "max_entry_basis", "max_entry_weights"]
        return {k: int(_lib().wq_points_info(self.h, i)) for i, k in enumerate(keys)}

    def get(self, what, stream=None):
        size = _lib().wq_points_size(self.h, what)
        out = torch.empty(size, dtype=_ARR_DTYPE[what], device="cuda")
        _check(_lib().wq_points_get(self.h, what, _ptr(out), _stream(stream)), "wq_points_get")
        return out

    def close(self):
        if self.h:
            _lib().wq_points_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Weights:
    """solve_weights: Gauss right-hand sides + truncated-SVD weights per family."""

    def __init__(self, mesh, points, fam_mask, tau=1e-12, stream=None):
        h = C.c_void_p()
        rep = SolveReport()
        _check(_lib().solve_weights(mesh.h, points.h, int(fam_mask), float(tau), _stream(stream), C.byref(h),
                                    C.byref(rep)), "solve_weights")
        self.h = h
        self.points = points
        self.fam_mask = fam_mask
        self.report = {k: getattr(rep, k) for k, _ in SolveReport._fields_}

    def weights(self, fam, stream=None):
        n = _lib().wq_points_size(self.points.h, ARR_QIDX)
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(_lib().wq_weights_get(self.h, fam, _ptr(out), _stream(stream)), "wq_weights_get")
        return out

    def rhs(self, fam, stream=None):
        out = torch.empty(self.points.nnz, dtype=torch.float64, device="cuda")
        _check(_lib().wq_rhs_get(self.h, fam, _ptr(out), _stream(stream)), "wq_rhs_get")
        return out

    def close(self):
        if self.h:
            _lib().wq_weights_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


GQ_MASS, GQ_STIFFNESS, GQ_BIHARMONIC = 0, 1, 2


class Gauss:
    """gauss_setup / assemble_gauss: element-wise 4 x 4 Gauss assembly on the WQ pattern."""

    def __init__(self, mesh, points, want_laplacian=False, stream=None):
        h = C.c_void_p()
        _check(_lib().gauss_setup(mesh.h, points.h, int(bool(want_laplacian)), _stream(stream), C.byref(h)),
               "gauss_setup")
        self.h = h
        self.points = points
        self.dim = mesh.dim
        self.size = int(_lib().wq_gauss_size(h))

    def x(self, stream=None):
        out = torch.empty(self.dim * self.size, dtype=torch.float64, device="cuda")
        _check(_lib().wq_gauss_get_x(self.h, _ptr(out), _stream(stream)), "wq_gauss_get_x")
        return out

    def assemble(self, kind, coef=None, out=None, stream=None):
        out = _out(self.points, out, WQ_FP64)
        if coef is not None:
            assert coef.dtype == torch.float64 and coef.numel() == self.size and coef.is_cuda and coef.is_contiguous()
        _check(_lib().assemble_gauss(self.h, int(kind), _ptr(coef), _ptr(out), _stream(stream)), "assemble_gauss")
        return out

    def close(self):
        if self.h:
            _lib().wq_gauss_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _out(points, out, prec):
    dt = torch.float64 if prec == WQ_FP64 else torch.float32
    if out is None:
        out = torch.empty(points.nnz, dtype=dt, device="cuda")
    assert out.dtype == dt and out.numel() == points.nnz and out.is_cuda and out.is_contiguous()
    return out


def _coef(points, c):
    if c is None:
        return None
    assert c.dtype == torch.float64 and c.numel() == points.n_points and c.is_cuda and c.is_contiguous()
    return c


def assemble_mass(points, weights, coef=None, out=None, prec=WQ_FP64, stream=None):
    out = _out(points, out, prec)
    _check(_lib().assemble_mass(points.h, weights.h, _ptr(_coef(points, coef)), _ptr(out), prec, _stream(stream)),
           "assemble_mass")
    return out


def assemble_stiffness(points, weights, coef=None, out=None, prec=WQ_FP64, stream=None):
    out = _out(points, out, prec)
    _check(_lib().assemble_stiffness(points.h, weights.h, _ptr(_coef(points, coef)), _ptr(out), prec,
                                     _stream(stream)), "assemble_stiffness")
    return out


def assemble_biharmonic(points, weights, coef=None, out=None, prec=WQ_FP64, stream=None):
    out = _out(points, out, prec)
    _check(_lib().assemble_biharmonic(points.h, weights.h, _ptr(_coef(points, coef)), _ptr(out), prec,
                                      _stream(stream)), "assemble_biharmonic")
    return out


def assemble_mass_stiffness(points, weights, c=None, k=None, mass_out=None, stiff_out=None, prec=WQ_FP64,
                            stream=None):
    mass_out = _out(points, mass_out, prec)
    stiff_out = _out(points, stiff_out, prec)
    _check(_lib().assemble_mass_stiffness(points.h, weights.h, _ptr(_coef(points, c)), _ptr(_coef(points, k)),
                                          _ptr(mass_out), _ptr(stiff_out), prec, _stream(stream)),
           "assemble_mass_stiffness")
    return mass_out, stiff_out


def _vec(t, n, dtype=torch.float64):
    assert t.dtype == dtype and t.numel() == n and t.is_cuda and t.is_contiguous()
    return t


def assemble_tangent(points, weights, T, Tdot, inv_theta_dt, k=(K_QUADRATIC, 1.0, 1.0), f=None, S_out=None,
                     R_out=None, stream=None, exact=False):
    """Eq. (36) tangent S (CSR values) and residual R at the fields T, Tdot; exact=True:
    the exact tangent of Eq. (34) (assemble_tangent_exact)."""
    n = points.n_rows
    S_out = _out(points, S_out, WQ_FP64)
    if R_out is None:
        R_out = torch.empty(n, dtype=torch.float64, device="cuda")
    _vec(T, n), _vec(Tdot, n), _vec(R_out, n)
    if f is not None:
        _vec(f, points.n_points)
    fn = _lib().assemble_tangent_exact if exact else _lib().assemble_tangent
    _check(fn(points.h, weights.h, _ptr(T), _ptr(Tdot), float(inv_theta_dt), Conductivity(*k), _ptr(f), _ptr(S_out),
              _ptr(R_out), WQ_FP64, _stream(stream)), "assemble_tangent")
    return S_out, R_out


def assemble_tangent_noalloc(points, weights, T, Tdot, inv_theta_dt, k=(K_QUADRATIC, 1.0, 1.0), f=None,
                             S_out=None, R_out=None, stream=None):
    """assemble_tangent through the entry point that allocates no device memory (its point
    fields sit in the library's fixed per-GPU array). S_out and R_out must be given."""
    n = points.n_rows
    assert S_out is not None and R_out is not None, "the caller provides the outputs"
    _vec(T, n), _vec(Tdot, n), _vec(R_out, n), _vec(S_out, points.nnz)
    if f is not None:
        _vec(f, points.n_points)
    _check(_lib().assemble_tangent_noalloc(points.h, weights.h, _ptr(T), _ptr(Tdot), float(inv_theta_dt),
                                           Conductivity(*k), _ptr(f), _ptr(S_out), _ptr(R_out), WQ_FP64,
                                           _stream(stream)),
           "assemble_tangent_noalloc")
    return S_out, R_out


def heat_step(points, weights, dirichlet, T, Tdot, dt, theta=1.0, k=(K_QUADRATIC, 1.0, 1.0), f=None, g=None,
              tol=1e-10, max_newton=50, cg_rtol=1e-6, max_cg=20000, S_out=None, stream=None,
              tangent=TANGENT_SYMMETRIC):
    """One time step of the nonlinear heat problem (Section 5.2); T and Tdot are
    updated in place. Returns the Newton/PCG report as a dict."""
    n = points.n_rows
    _vec(dirichlet, n, torch.uint8), _vec(T, n), _vec(Tdot, n)
    if f is not None:
        _vec(f, points.n_points)
    if g is not None:
        _vec(g, n)
    S_out = _out(points, S_out, WQ_FP64)
    hp = HeatParams(float(dt), float(theta), Conductivity(*k), float(tol), int(max_newton), float(cg_rtol),
                    int(max_cg), int(tangent))
    rep = HeatReport()
    _check(_lib().wq_heat_step(points.h, weights.h, C.byref(hp), _ptr(dirichlet), _ptr(g), _ptr(f), _ptr(T),
                               _ptr(Tdot), _ptr(S_out), C.byref(rep), _stream(stream)), "wq_heat_step")
    return {k_: getattr(rep, k_) for k_, _ in HeatReport._fields_}


def _mesh_desc(fx, keep):
    keep.update({
        "face_vtx": np.ascontiguousarray(fx["face_vtx"], dtype=np.int32),
        "split": np.ascontiguousarray(fx["split"], dtype=np.uint8),
        "ext_ptr": np.ascontiguousarray(fx["ext_ptr"], dtype=np.int64),
        "ext_fn": np.ascontiguousarray(fx["ext_fn"], dtype=np.int32),
        "coef_ptr": np.ascontiguousarray(fx["coef_ptr"], dtype=np.int64),
        "coef": np.ascontiguousarray(fx["coef"], dtype=np.float64),
        "ctrl": np.ascontiguousarray(fx["ctrl"], dtype=np.float64),
    })
    return MeshDesc(int(fx["nv"]), int(len(keep["face_vtx"])), int(fx["n_fn"]),
                    *[C.c_void_p(keep[n].ctypes.data) for n in ("face_vtx", "split", "ext_ptr", "ext_fn", "coef_ptr",
                                                                "coef", "ctrl")], int(keep["ctrl"].shape[1]))


class Server:
    """wq_server_*: requests of (mesh, prescribed DOFs, heat parameters, steps) served
    with HBM-budget admission on `slots` concurrent streams."""

    def __init__(self, hbm_budget_bytes, slots):
        h = C.c_void_p()
        _check(_lib().wq_server_start(int(hbm_budget_bytes), int(slots), C.byref(h)), "wq_server_start")
        self.h = h
        self._out = {}

    def submit(self, fx, dirichlet, dt, n_steps, theta=1.0, k=(K_QUADRATIC, 1.0, 1.0), source=SOURCE_MANUFACTURED,
               lam=5.0, tol=1e-10, max_newton=50, cg_rtol=1e-6, max_cg=20000, tangent=TANGENT_SYMMETRIC,
               reuse_setup=True):
        keep = {}
        desc = _mesh_desc(fx, keep)
        keep["dirichlet"] = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        hp = HeatParams(float(dt), float(theta), Conductivity(*k), float(tol), int(max_newton), float(cg_rtol),
                        int(max_cg), int(tangent))
        req = Request(desc, C.c_void_p(keep["dirichlet"].ctypes.data), hp, int(n_steps), int(source), float(lam),
                      1 if reuse_setup else 0)
        T = np.zeros(int(fx["n_fn"]), dtype=np.float64)
        ticket = C.c_int64()
        _check(_lib().wq_server_submit(self.h, C.byref(req), C.c_void_p(T.ctypes.data), C.byref(ticket)),
               "wq_server_submit")
        self._out[ticket.value] = T
        return ticket.value

    def set_join(self, max_meshes, max_rows=1 << 15):
        """Requests queued together with the same parameters run as one union of up to
        `max_meshes` meshes and `max_rows` rows (1 mesh: each alone)."""
        _check(_lib().wq_server_set_join(self.h, int(max_meshes), int(max_rows)), "wq_server_set_join")

    def poll(self, ticket, wait=True):
        """None while pending; else (T, result dict)."""
        res = Result()
        st = _lib().wq_server_poll(self.h, int(ticket), 1 if wait else 0, C.byref(res))
        if st < 0:
            raise WQError(st, "wq_server_poll")
        if st == 0:
            return None
        return self._out.pop(ticket), {k_: getattr(res, k_) for k_, _ in Result._fields_}

    def close(self):
        if self.h:
            _lib().wq_server_stop(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Borrowed:
    """Points / weights handle owned by a batch (not destroyed by the wrapper)."""

    def __init__(self, h, **kw):
        self.h = h
        self.__dict__.update(kw)

    def get(self, what, stream=None):
        return Points.get(self, what, stream)

    def weights(self, fam, stream=None):
        return Weights.weights(self, fam, stream)

    def rhs(self, fam, stream=None):
        return Weights.rhs(self, fam, stream)

    def info(self):
        return Points.info(self)


class Batch:
    """wq_batch_*: many meshes joined into one union and processed by one set of launches."""

    def __init__(self, fixtures):
        self._keep = [dict() for _ in fixtures]
        descs = (MeshDesc * len(fixtures))(*[_mesh_desc(fx, k) for fx, k in zip(fixtures, self._keep)])
        h = C.c_void_p()
        _check(_lib().wq_batch_create(descs, len(fixtures), C.byref(h)), "wq_batch_create")
        self.h = h
        self.n_meshes = len(fixtures)
        self.points = self.weights = None

    def build(self, fam_mask, tau=1e-12, stream=None):
        rep = SolveReport()
        _check(_lib().wq_batch_build(self.h, int(fam_mask), float(tau), _stream(stream), C.byref(rep)),
               "wq_batch_build")
        self.report = {k: getattr(rep, k) for k, _ in SolveReport._fields_}
        ph = C.c_void_p(_lib().wq_batch_points(self.h))
        n = _lib().wq_points_size(ph, ARR_ROW_PTR) - 1
        nnz = _lib().wq_points_size(ph, ARR_COL)
        npt = _lib().wq_points_size(ph, ARR_X) // 2
        self.points = _Borrowed(ph, n_rows=n, nnz=nnz, n_points=npt)
        self.weights = _Borrowed(C.c_void_p(_lib().wq_batch_weights(self.h)), points=self.points)
        return self

    def info(self, k):
        v = [C.c_int64() for _ in range(6)]
        _check(_lib().wq_batch_info(self.h, int(k), *[C.byref(x) for x in v]), "wq_batch_info")
        return dict(zip(("row0", "n_rows", "nnz0", "nnz", "pt0", "n_points"), [x.value for x in v]))

    def graph_assemble(self, c, k, mass_out, stiff_out, prec=WQ_FP64, stream=None):
        _check(_lib().wq_batch_graph_assemble(self.h, _ptr(c), _ptr(k), _ptr(mass_out), _ptr(stiff_out), int(prec),
                                              _stream(stream)), "wq_batch_graph_assemble")

    def close(self):
        if self.h:
            _lib().wq_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_assembly(points, weights, stream=None):
    """Pick the assembly's XCD chunk length on `points` by measurement; returns (chunk, ms)."""
    ch, ms = C.c_int32(), C.c_double()
    _check(_lib().wq_autotune_assembly(points.h, weights.h, _stream(stream), C.byref(ch), C.byref(ms)),
           "wq_autotune_assembly")
    return ch.value, ms.value


def autotune_tiles(points, weights, stream=None):
    """Pick the assembly's tile work cap and XCD chunk length on `points` by measurement;
    returns (step cap, chunk, ms)."""
    cap, ch, ms = C.c_int32(), C.c_int32(), C.c_double()
    _check(_lib().wq_autotune_tiles(points.h, weights.h, _stream(stream), C.byref(cap), C.byref(ch), C.byref(ms)),
           "wq_autotune_tiles")
    return cap.value, ch.value, ms.value


def timing_enable(on=True):
    """Record HIP events around the library's main kernels (measurement aid)."""
    _lib().wq_timing_enable(1 if on else 0)


def set_side_streams(n):
    """Streams for the independent launches within one call (1: all on the caller's stream)."""
    _check(_lib().wq_set_side_streams(int(n)), "wq_set_side_streams")


def timings(cap=4096):
    """[(kernel name, ms, work units)] recorded since the last call (synchronises)."""
    buf = (Timing * cap)()
    n = _lib().wq_timings(buf, cap)
    return [(buf[i].name.decode(), buf[i].ms, buf[i].work) for i in range(n)]
