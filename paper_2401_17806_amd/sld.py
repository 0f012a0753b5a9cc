"""Thin ctypes binding of libsld.so (the C ABI declared in include/sld.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device buffers are torch tensors (float64, contiguous, on the
handle's device); the current torch stream of that device is passed as the
HIP stream.  Shapes, dtypes and devices are checked here, on the host,
before any launch.  There is no fallback: if the library is missing the
import fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch first: its HIP runtime is then the one libsld.so binds to, so the streams and device
# pointers torch hands over belong to the same runtime as the library's own calls
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsld.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2401_17806_amd.build` "
        "(hipcc, gfx950); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

_c_dp = ctypes.POINTER(ctypes.c_double)
_c_ip = ctypes.POINTER(ctypes.c_int32)
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


class sld_cg_params(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double), ("maxit", _i32),
                ("warm_start", _i32), ("graph_block", _i32), ("profile", _i32),
                ("precision", _i32), ("max_outer", _i32), ("engine", _i32),
                ("pipelined", _i32)]


class sld_cg_report(ctypes.Structure):
    _fields_ = [("iters", _i32), ("converged", _i32), ("rel_res", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("seconds", ctypes.c_double),
                ("step_us", ctypes.c_double), ("timed_iters", _i32), ("outer_iters", _i32)]


class sld_imex_params(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("R", _i32), ("pressure", sld_cg_params),
                ("viscous", sld_cg_params)]


class sld_imex_report(ctypes.Structure):
    _fields_ = [("pressure", sld_cg_report), ("viscous", sld_cg_report * 2),
                ("seconds", ctypes.c_double)]


class sld_boussinesq_params(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("kappa", ctypes.c_double), ("gbeta", ctypes.c_double),
                ("R", _i32), ("pressure", sld_cg_params), ("viscous", sld_cg_params)]


class sld_boussinesq_report(ctypes.Structure):
    _fields_ = [("pressure", sld_cg_report), ("viscous", sld_cg_report * 2),
                ("temperature", sld_cg_report), ("seconds", ctypes.c_double)]


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_lib.sld_last_error.restype = ctypes.c_char_p
_lib.sld_last_error.argtypes = []
_sig("sld_abi_version", [], _i32)
_sig("sld_mesh_create", [_c_dp, _i64, _c_ip, _i64, _c_dp, _i32, ctypes.POINTER(_vp)])
_sig("sld_mesh_counts", [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)])
_sig("sld_mesh_edges", [_vp, _c_ip, _c_ip, _c_ip, _c_ip])
_sig("sld_mesh_destroy", [_vp], None)
_sig("sld_disc_create", [_vp, _i32, ctypes.c_uint32, ctypes.POINTER(_vp)])
_sig("sld_disc_info", [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)])
_sig("sld_main_nodes", [_vp, _c_dp])
_sig("sld_dual_nodes", [_vp, _c_dp])
_sig("sld_main_weights", [_vp, _c_dp])
_sig("sld_disc_destroy", [_vp], None)
_sig("sld_schur_apply", [_vp, _vp, _vp, _vp])
_sig("sld_schur_apply_mx", [_vp, _vp, _vp, _i32, _vp])
_sig("sld_gradient", [_vp, _vp, _vp, _vp])
_sig("sld_divergence", [_vp, _vp, _vp, _vp])
_sig("sld_pressure_rhs", [_vp, _vp, ctypes.c_double, _vp, _vp])
_sig("sld_velocity_correct", [_vp, _vp, _vp, ctypes.c_double, _vp, _vp])
_sig("sld_cg_solve", [_vp, _vp, _vp, ctypes.POINTER(sld_cg_params),
                      ctypes.POINTER(sld_cg_report), _vp])
_sig("sld_cg_solve_static", [_vp, _vp, _vp, ctypes.POINTER(sld_cg_params),
                             ctypes.POINTER(sld_cg_report), _vp])
_sig("sld_disc_footprint", [_vp, ctypes.POINTER(ctypes.c_uint64)])
_sig("sld_ref_operator", [_vp, _i32, _i32, _c_dp, _i64, ctypes.POINTER(_i64)])
_sig("sld_sl_advect", [_vp, _vp, _vp, _i32, ctypes.c_double, _vp, _vp])
_sig("sld_dual_to_main", [_vp, _vp, _i32, _vp, _vp])
_sig("sld_main_to_dual", [_vp, _vp, _i32, _vp, _vp])
_sig("sld_viscous_solve", [_vp, _vp, ctypes.c_double, _vp, _vp, _vp,
                           ctypes.POINTER(sld_cg_params), ctypes.POINTER(sld_cg_report), _vp])
_sig("sld_state_create", [_vp, ctypes.POINTER(_vp)])
_sig("sld_state_destroy", [_vp], None)
_sig("sld_imex_step", [_vp, ctypes.POINTER(sld_imex_params), ctypes.c_double, _vp, _vp,
                       ctypes.POINTER(sld_imex_report), _vp])
_sig("sld_boussinesq_step", [_vp, ctypes.POINTER(sld_boussinesq_params), ctypes.c_double, _vp,
                             _vp, _vp, _vp, _vp, ctypes.POINTER(sld_boussinesq_report), _vp])
_sig("sld_server_create", [_i32, ctypes.c_uint64, _i32, ctypes.POINTER(_vp)])
_sig("sld_server_submit", [_vp, _vp, _vp, _vp, ctypes.POINTER(sld_cg_params), _vp,
                           ctypes.POINTER(ctypes.c_uint64)])
_sig("sld_server_submit_imex", [_vp, _vp, ctypes.POINTER(sld_imex_params), ctypes.c_double, _vp,
                                _vp, _vp, ctypes.POINTER(ctypes.c_uint64)])
_sig("sld_server_poll", [_vp, ctypes.c_uint64, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                         ctypes.POINTER(sld_cg_report)])
_sig("sld_server_stats", [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                          ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)])
_sig("sld_server_destroy", [_vp], None)

EXPORTED = [
    "sld_last_error", "sld_abi_version", "sld_mesh_create", "sld_mesh_counts", "sld_mesh_edges",
    "sld_mesh_destroy", "sld_disc_create", "sld_disc_info", "sld_main_nodes", "sld_dual_nodes",
    "sld_main_weights", "sld_disc_destroy", "sld_schur_apply", "sld_schur_apply_mx", "sld_gradient",
    "sld_divergence",
    "sld_pressure_rhs", "sld_velocity_correct", "sld_cg_solve", "sld_cg_solve_static",
    "sld_disc_footprint",
    "sld_sl_advect", "sld_ref_operator", "sld_dual_to_main", "sld_main_to_dual",
    "sld_viscous_solve", "sld_state_create", "sld_state_destroy", "sld_imex_step",
    "sld_boussinesq_step",
    "sld_server_create", "sld_server_submit", "sld_server_submit_imex", "sld_server_poll",
    "sld_server_stats",
    "sld_server_destroy",
]

STATUS = {0: "SLD_OK", 1: "SLD_E_INVALID", 2: "SLD_E_MESH", 3: "SLD_E_NOMEM", 4: "SLD_E_HIP",
          5: "SLD_E_NOCONV", 6: "SLD_E_BREAKDOWN", 7: "SLD_E_BUDGET"}


class SldError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(status):
    if status != 0:
        raise SldError(status, _lib.sld_last_error().decode(errors="replace"))


def sld_last_error() -> str:
    return _lib.sld_last_error().decode(errors="replace")


def sld_abi_version() -> int:
    return int(_lib.sld_abi_version())


def _host_f64(a, shape_tail=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a


def _dptr(a):
    return a.ctypes.data_as(_c_dp)


# ---------------------------------------------------------------- raw C-named wrappers
def sld_mesh_create(xy, tri, period=None, device: int = 0):
    xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64))
    tri = np.ascontiguousarray(np.asarray(tri, dtype=np.int32))
    if xy.ndim != 2 or xy.shape[1] != 2 or tri.ndim != 2 or tri.shape[1] != 3:
        raise ValueError("xy must be [nv, 2] and tri [ne, 3]")
    per = None if period is None else np.ascontiguousarray(np.asarray(period, dtype=np.float64))
    if per is not None and per.shape != (2,):
        raise ValueError("period must have shape (2,)")
    h = _vp()
    _check(_lib.sld_mesh_create(_dptr(xy), xy.shape[0], tri.ctypes.data_as(_c_ip), tri.shape[0],
                                None if per is None else _dptr(per), int(device), ctypes.byref(h)))
    return h


def sld_mesh_counts(h):
    ne, nd, nv = _i64(), _i64(), _i64()
    _check(_lib.sld_mesh_counts(h, ctypes.byref(ne), ctypes.byref(nd), ctypes.byref(nv)))
    return ne.value, nd.value, nv.value


def sld_mesh_edges(h):
    _, nd, _ = sld_mesh_counts(h)
    arrs = [np.empty(nd, dtype=np.int32) for _ in range(4)]
    _check(_lib.sld_mesh_edges(h, *[a.ctypes.data_as(_c_ip) for a in arrs]))
    return tuple(arrs)


def sld_mesh_destroy(h):
    _lib.sld_mesh_destroy(h)


def sld_disc_create(mesh_h, p: int):
    h = _vp()
    _check(_lib.sld_disc_create(mesh_h, int(p), 0, ctypes.byref(h)))
    return h


def sld_disc_info(h):
    p, nphi, npsi = _i32(), _i32(), _i32()
    _check(_lib.sld_disc_info(h, ctypes.byref(p), ctypes.byref(nphi), ctypes.byref(npsi)))
    return p.value, nphi.value, npsi.value


def sld_disc_destroy(h):
    _lib.sld_disc_destroy(h)


ENGINES = {"auto": 0, "valu": 1, "mfma": 2}
PIPELINED = {"auto": 0, "classic": 1, "pipelined": 2}


def make_params(rtol=1e-12, maxit=100000, warm_start=False, graph_block=32, profile=False,
                precision="fp64", inner_rtol=0.5, max_outer=1000, engine="auto",
                algorithm="auto"):
    if precision not in ("fp64", "mixed"):
        raise ValueError("precision must be 'fp64' or 'mixed'")
    if engine not in ENGINES:
        raise ValueError("engine must be 'auto' (the library's choice), 'valu' or 'mfma'")
    if algorithm not in PIPELINED:
        raise ValueError("algorithm must be 'auto' (the library's choice), 'classic' or "
                         "'pipelined'")
    return sld_cg_params(float(rtol), float(inner_rtol), int(maxit), int(bool(warm_start)),
                         int(graph_block), int(bool(profile)), 1 if precision == "mixed" else 0,
                         int(max_outer), ENGINES[engine], PIPELINED[algorithm])


def report_dict(rep, st):
    return {"iters": rep.iters, "converged": bool(rep.converged), "rel_res": rep.rel_res,
            "rel_res_true": rep.rel_res_true, "seconds": rep.seconds, "step_us": rep.step_us,
            "timed_iters": rep.timed_iters, "outer_iters": rep.outer_iters,
            "status": STATUS.get(st, st)}


class Mesh:
    """Owner of an sld_mesh handle."""

    def __init__(self, xy, tri, period=None, device: int = 0):
        self.device = int(device)
        self.handle = sld_mesh_create(xy, tri, period, device)
        self.ne, self.nd, self.nv = sld_mesh_counts(self.handle)

    def edges(self):
        return sld_mesh_edges(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            sld_mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Disc:
    """Owner of an sld_disc handle; operator entry points take torch device tensors."""

    def __init__(self, mesh: Mesh, p: int):
        self.mesh = mesh
        self.handle = sld_disc_create(mesh.handle, p)
        self.p, self.nphi, self.npsi = sld_disc_info(self.handle)
        self.main_shape = (mesh.ne, self.nphi)
        self.dual_shape = (mesh.nd, 2, self.npsi)

    # -------------------------------------------------------- host queries
    def main_nodes(self):
        out = np.empty((self.mesh.ne, self.nphi, 2))
        _check(_lib.sld_main_nodes(self.handle, _dptr(out)))
        return out

    def dual_nodes(self):
        out = np.empty((self.mesh.nd, self.npsi, 2))
        _check(_lib.sld_dual_nodes(self.handle, _dptr(out)))
        return out

    def main_weights(self):
        out = np.empty((self.mesh.ne, self.nphi))
        _check(_lib.sld_main_weights(self.handle, _dptr(out)))
        return out

    # -------------------------------------------------------- device helpers
    def _dev(self, t, shape, name):
        import torch
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.float64 or not t.is_cuda or t.device.index != self.mesh.device:
            raise ValueError(f"{name} must be float64 on cuda:{self.mesh.device}")
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {tuple(shape)}, got {tuple(t.shape)}")
        return _vp(t.data_ptr())

    def _stream(self, stream):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.mesh.device)
        return _vp(s.cuda_stream)

    def _new(self, shape):
        import torch
        return torch.empty(shape, dtype=torch.float64, device=f"cuda:{self.mesh.device}")

    # -------------------------------------------------------- operators
    def sld_schur_apply(self, p, out=None, stream=None):
        out = self._new(self.main_shape) if out is None else out
        _check(_lib.sld_schur_apply(self.handle, self._dev(p, self.main_shape, "p"),
                                    self._dev(out, self.main_shape, "Kp"), self._stream(stream)))
        return out

    def sld_schur_apply_mx(self, p, engine="f64", out=None, stream=None):
        """K p on the matrix cores: engine "f64" (float64 tensors) or "bf16x3" (float32)."""
        import torch
        code = {"f64": 0, "bf16x3": 1}[engine]
        dt = torch.float64 if code == 0 else torch.float32
        if out is None:
            out = torch.empty(self.main_shape, dtype=dt, device=f"cuda:{self.mesh.device}")
        for name, t in (("p", p), ("Kp", out)):
            if (not isinstance(t, torch.Tensor) or t.dtype != dt or not t.is_cuda
                    or t.device.index != self.mesh.device or tuple(t.shape) != self.main_shape
                    or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous {dt} tensor {self.main_shape} "
                                 f"on cuda:{self.mesh.device}")
        _check(_lib.sld_schur_apply_mx(self.handle, _vp(p.data_ptr()), _vp(out.data_ptr()), code,
                                       self._stream(stream)))
        return out

    def sld_gradient(self, p, out=None, stream=None):
        out = self._new(self.dual_shape) if out is None else out
        _check(_lib.sld_gradient(self.handle, self._dev(p, self.main_shape, "p"),
                                 self._dev(out, self.dual_shape, "g"), self._stream(stream)))
        return out

    def sld_divergence(self, v, out=None, stream=None):
        out = self._new(self.main_shape) if out is None else out
        _check(_lib.sld_divergence(self.handle, self._dev(v, self.dual_shape, "v"),
                                   self._dev(out, self.main_shape, "out"), self._stream(stream)))
        return out

    def sld_pressure_rhs(self, v_star, scale, out=None, stream=None):
        out = self._new(self.main_shape) if out is None else out
        _check(_lib.sld_pressure_rhs(self.handle, self._dev(v_star, self.dual_shape, "v_star"),
                                     float(scale), self._dev(out, self.main_shape, "b"),
                                     self._stream(stream)))
        return out

    def sld_velocity_correct(self, v_star, p, coef, out=None, stream=None):
        out = self._new(self.dual_shape) if out is None else out
        _check(_lib.sld_velocity_correct(self.handle, self._dev(v_star, self.dual_shape, "v_star"),
                                         self._dev(p, self.main_shape, "p"), float(coef),
                                         self._dev(out, self.dual_shape, "v"), self._stream(stream)))
        return out

    def footprint(self) -> int:
        v = ctypes.c_uint64()
        _check(_lib.sld_disc_footprint(self.handle, ctypes.byref(v)))
        return int(v.value)

    REF_OPERATORS = {"S": 0, "Sh": 1, "E": 2, "Pt": 3, "C": 4, "M1": 5, "w": 6,
                     "sl_points": 7, "sl_proj": 8, "Mref": 9, "Ldm": 10}

    def sld_ref_operator(self, which: str, alpha: int = 0) -> np.ndarray:
        """Host copy of a reference operator (flat float64; see include/sld.h for shapes)."""
        code = self.REF_OPERATORS[which]
        cnt = _i64()
        _check(_lib.sld_ref_operator(self.handle, code, int(alpha), None, 0, ctypes.byref(cnt)))
        out = np.empty(cnt.value, dtype=np.float64)
        _check(_lib.sld_ref_operator(self.handle, code, int(alpha),
                                     out.ctypes.data_as(_c_dp), cnt.value, ctypes.byref(cnt)))
        return out

    def sld_sl_advect(self, vbar, q, dt, out=None, stream=None):
        """q [ne, nc, N_phi] advected over dt by the velocity vbar [ne, 2, N_phi]."""
        import torch
        if q.dim() != 3 or q.shape[0] != self.mesh.ne or q.shape[2] != self.nphi:
            raise ValueError(f"q must be [{self.mesh.ne}, nc, {self.nphi}]")
        nc = int(q.shape[1])
        self._dev(vbar, (self.mesh.ne, 2, self.nphi), "vbar")
        self._dev(q, tuple(q.shape), "q")
        if out is None:
            out = torch.empty_like(q)
        self._dev(out, tuple(q.shape), "out")
        _check(_lib.sld_sl_advect(self.handle, _vp(vbar.data_ptr()), _vp(q.data_ptr()), nc,
                                  float(dt), _vp(out.data_ptr()), self._stream(stream)))
        return out

    def sld_cg_solve(self, b, p=None, rtol=1e-12, maxit=100000, warm_start=False,
                     graph_block=32, profile=False, precision="fp64", inner_rtol=0.5,
                     max_outer=1000, stream=None, engine="auto", algorithm="auto"):
        """Solve K p = b (gauge int p = 0).  precision: "fp64" or "mixed"; engine: "auto" (the
        library's choice), "valu" (vector units) or "mfma" (matrix cores where the mesh has no
        walls); algorithm (FP64 pressure iterations): "auto", "classic" or "pipelined" (meshes of
        one tile per block of the CG grid)."""
        p = self._new(self.main_shape) if p is None else p
        prm = make_params(rtol, maxit, warm_start, graph_block, profile, precision, inner_rtol,
                          max_outer, engine, algorithm)
        rep = sld_cg_report()
        st = _lib.sld_cg_solve(self.handle, self._dev(b, self.main_shape, "b"),
                               self._dev(p, self.main_shape, "p"), ctypes.byref(prm),
                               ctypes.byref(rep), self._stream(stream))
        report = report_dict(rep, st)
        if st not in (0, 5):
            _check(st)
        return p, report

    def sld_cg_solve_static(self, b, p=None, rtol=1e-12, maxit=100000, warm_start=False,
                            graph_block=32, stream=None):
        """sld_cg_solve in FP64 with its workspace in the library's static device array (no
        device allocation in the call; p must be given to allocate nothing at all)."""
        p = self._new(self.main_shape) if p is None else p
        prm = make_params(rtol, maxit, warm_start, graph_block, False, "fp64", 0.5, 1)
        rep = sld_cg_report()
        st = _lib.sld_cg_solve_static(self.handle, self._dev(b, self.main_shape, "b"),
                                      self._dev(p, self.main_shape, "p"), ctypes.byref(prm),
                                      ctypes.byref(rep), self._stream(stream))
        report = report_dict(rep, st)
        if st not in (0, 5):
            _check(st)
        return p, report

    def sld_dual_to_main(self, v, out=None, stream=None):
        """L2 projection of a dual field v [nd, nc, N_psi] onto the main space (eq. d2m)."""
        if v.dim() != 3 or v.shape[0] != self.mesh.nd or v.shape[2] != self.npsi:
            raise ValueError(f"v must be [{self.mesh.nd}, nc, {self.npsi}]")
        nc = int(v.shape[1])
        shape = (self.mesh.ne, nc, self.nphi)
        out = self._new(shape) if out is None else out
        _check(_lib.sld_dual_to_main(self.handle, self._dev(v, tuple(v.shape), "v"), nc,
                                     self._dev(out, shape, "out"), self._stream(stream)))
        return out

    def sld_main_to_dual(self, v, out=None, stream=None):
        """L2 projection of a main field v [ne, nc, N_phi] onto the dual space (eq. m2d)."""
        if v.dim() != 3 or v.shape[0] != self.mesh.ne or v.shape[2] != self.nphi:
            raise ValueError(f"v must be [{self.mesh.ne}, nc, {self.nphi}]")
        nc = int(v.shape[1])
        shape = (self.mesh.nd, nc, self.npsi)
        out = self._new(shape) if out is None else out
        _check(_lib.sld_main_to_dual(self.handle, self._dev(v, tuple(v.shape), "v"), nc,
                                     self._dev(out, shape, "out"), self._stream(stream)))
        return out

    def sld_viscous_solve(self, f, c, x=None, wall_dirichlet=None, wall_values=None, rtol=1e-12,
                          maxit=100000, graph_block=32, stream=None):
        """x with (Mbar - c K_W) x = Mbar f + c G_b (FP64 CG).  wall_dirichlet: uint8 device
        tensor [nd] flagging Dirichlet wall edges; wall_values: float64 [nd, p+1] data."""
        import torch
        x = self._new(self.main_shape) if x is None else x
        mask_p = _vp(0)
        if wall_dirichlet is not None:
            if (wall_dirichlet.dtype != torch.uint8 or not wall_dirichlet.is_cuda or
                    tuple(wall_dirichlet.shape) != (self.mesh.nd,) or
                    not wall_dirichlet.is_contiguous()):
                raise ValueError(f"wall_dirichlet must be a contiguous uint8 cuda tensor [{self.mesh.nd}]")
            mask_p = _vp(wall_dirichlet.data_ptr())
        vals_p = _vp(0)
        if wall_values is not None:
            vals_p = self._dev(wall_values, (self.mesh.nd, self.p + 1), "wall_values")
        prm = make_params(rtol, maxit, False, graph_block)
        rep = sld_cg_report()
        st = _lib.sld_viscous_solve(self.handle, self._dev(f, self.main_shape, "f"), float(c),
                                    mask_p, vals_p, self._dev(x, self.main_shape, "x"),
                                    ctypes.byref(prm), ctypes.byref(rep), self._stream(stream))
        report = report_dict(rep, st)
        if st not in (0, 5):
            _check(st)
        return x, report

    def close(self):
        if getattr(self, "handle", None):
            sld_disc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class State:
    """Owner of an sld_state handle (IMEX step workspace); keeps its Disc alive."""

    def __init__(self, disc: Disc):
        self.disc = disc
        h = _vp()
        _check(_lib.sld_state_create(disc.handle, ctypes.byref(h)))
        self.handle = h

    def sld_imex_step(self, v, p, dt, nu, R=0, rtol=1e-12, visc_rtol=1e-12, maxit=200000,
                      graph_block=32, warm_start=True, precision="fp64", profile=False,
                      stream=None):
        """One IMEX step in place: v [nd, 2, N_psi] at t -> t + dt; p [ne, N_phi] <- pressure."""
        d = self.disc
        prm = sld_imex_params(float(nu), int(R),
                              make_params(rtol, maxit, warm_start, graph_block,
                                          profile and precision == "fp64", precision),
                              make_params(visc_rtol, maxit, True, graph_block))
        rep = sld_imex_report()
        st = _lib.sld_imex_step(self.handle, ctypes.byref(prm), float(dt),
                                d._dev(v, d.dual_shape, "v"), d._dev(p, d.main_shape, "p"),
                                ctypes.byref(rep), d._stream(stream))
        out = {"pressure": report_dict(rep.pressure, st),
               "viscous": [report_dict(rep.viscous[k], st) for k in range(2)],
               "seconds": rep.seconds, "status": STATUS.get(st, st)}
        if st not in (0, 5):
            _check(st)
        return out

    def sld_boussinesq_step(self, v, T, p, dt, nu, kappa, gbeta, temp_dirichlet=None,
                            temp_values=None, R=0, rtol=1e-12, visc_rtol=1e-12, maxit=200000,
                            graph_block=32, warm_start=True, precision="fp64", stream=None):
        """One Boussinesq step in place: v [nd, 2, N_psi], T [ne, N_phi]; p [ne, N_phi] out.
        temp_dirichlet: uint8 cuda tensor [nd]; temp_values: float64 [nd, p+1]."""
        import torch
        d = self.disc
        mask_p = _vp(0)
        if temp_dirichlet is not None:
            if (temp_dirichlet.dtype != torch.uint8 or not temp_dirichlet.is_cuda or
                    tuple(temp_dirichlet.shape) != (d.mesh.nd,) or
                    not temp_dirichlet.is_contiguous()):
                raise ValueError(f"temp_dirichlet must be a contiguous uint8 cuda tensor [{d.mesh.nd}]")
            mask_p = _vp(temp_dirichlet.data_ptr())
        vals_p = _vp(0) if temp_values is None else d._dev(temp_values, (d.mesh.nd, d.p + 1),
                                                           "temp_values")
        prm = sld_boussinesq_params(float(nu), float(kappa), float(gbeta), int(R),
                                    make_params(rtol, maxit, warm_start, graph_block, False,
                                                precision),
                                    make_params(visc_rtol, maxit, True, graph_block))
        rep = sld_boussinesq_report()
        st = _lib.sld_boussinesq_step(self.handle, ctypes.byref(prm), float(dt), mask_p, vals_p,
                                      d._dev(v, d.dual_shape, "v"), d._dev(T, d.main_shape, "T"),
                                      d._dev(p, d.main_shape, "p"), ctypes.byref(rep),
                                      d._stream(stream))
        out = {"pressure": report_dict(rep.pressure, st),
               "viscous": [report_dict(rep.viscous[k], st) for k in range(2)],
               "temperature": report_dict(rep.temperature, st),
               "seconds": rep.seconds, "status": STATUS.get(st, st)}
        if st not in (0, 5):
            _check(st)
        return out

    def close(self):
        if getattr(self, "handle", None):
            _lib.sld_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Owner of an sld_server handle (continuous batching of solves, see include/sld.h)."""

    def __init__(self, device: int = 0, budget_bytes: int = 16 << 30, workers: int = 4):
        self.device = int(device)
        self.handle = _vp()
        _check(_lib.sld_server_create(self.device, int(budget_bytes), int(workers),
                                      ctypes.byref(self.handle)))
        self._keep = {}

    def sld_server_submit(self, disc: Disc, b, p, stream=None, **params):
        prm = make_params(**params)
        t = ctypes.c_uint64()
        _check(_lib.sld_server_submit(self.handle, disc.handle, disc._dev(b, disc.main_shape, "b"),
                                      disc._dev(p, disc.main_shape, "p"), ctypes.byref(prm),
                                      disc._stream(stream), ctypes.byref(t)))
        self._keep[t.value] = (b, p)  # buffers stay alive until the ticket completes
        return t.value

    def sld_server_submit_imex(self, state: "State", v, p, dt, nu, R=0, rtol=1e-12,
                               visc_rtol=1e-12, maxit=200000, graph_block=32, warm_start=True,
                               precision="fp64", stream=None):
        d = state.disc
        prm = sld_imex_params(float(nu), int(R),
                              make_params(rtol, maxit, warm_start, graph_block, False, precision),
                              make_params(visc_rtol, maxit, True, graph_block))
        t = ctypes.c_uint64()
        _check(_lib.sld_server_submit_imex(self.handle, state.handle, ctypes.byref(prm), float(dt),
                                           d._dev(v, d.dual_shape, "v"), d._dev(p, d.main_shape, "p"),
                                           d._stream(stream), ctypes.byref(t)))
        self._keep[t.value] = (state, v, p)  # alive until the ticket completes
        return t.value

    def sld_server_poll(self, ticket: int, wait: bool = False):
        done, st = _i32(), _i32()
        rep = sld_cg_report()
        _check(_lib.sld_server_poll(self.handle, ctypes.c_uint64(ticket), int(bool(wait)),
                                    ctypes.byref(done), ctypes.byref(st), ctypes.byref(rep)))
        if not done.value:
            return None
        self._keep.pop(ticket, None)
        return report_dict(rep, st.value)

    def sld_server_stats(self):
        q, r = _i32(), _i32()
        b, c = ctypes.c_uint64(), ctypes.c_uint64()
        _check(_lib.sld_server_stats(self.handle, ctypes.byref(q), ctypes.byref(r), ctypes.byref(b),
                                     ctypes.byref(c)))
        return {"queued": q.value, "running": r.value, "in_flight_bytes": b.value,
                "completed": c.value}

    def close(self):
        if getattr(self, "handle", None):
            _lib.sld_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
