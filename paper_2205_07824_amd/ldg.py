"""Thin ctypes binding of the gfx950 LDG library (libldg.so).

Argument marshalling only: every step of the residual / Jacobian-vector product
/ preconditioner / GMRES / Newton path runs in the library's HIP kernels.  Torch
supplies device memory and the current stream.  The names mirror the C ABI
declared in include/ldg.h.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldg.so")

LDG_OK, LDG_EINVAL, LDG_EUNSUPPORTED, LDG_EDEVICE, LDG_ENOMEM, LDG_ENOCONV, LDG_EBREAKDOWN = range(7)
FP64, FP32, BF16_MFMA, FP16_MFMA, JVP_FD, BF16, FP16 = range(7)
MODEL_POISSON, MODEL_CONVDIFF, MODEL_EULER, MODEL_NS, MODEL_USER = range(5)
BC_DIRICHLET, BC_NEUMANN, BC_EXTRAP = range(3)

_STATUS = {0: "OK", 1: "EINVAL", 2: "EUNSUPPORTED", 3: "EDEVICE", 4: "ENOMEM", 5: "ENOCONV", 6: "EBREAKDOWN"}


class LDGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Time(C.Structure):
    _fields_ = [("a0", C.c_double), ("r1", C.c_void_p), ("c1", C.c_double), ("r2", C.c_void_p), ("c2", C.c_double)]


class _ModelDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("ncu", C.c_int), ("nmu", C.c_int), ("mu", C.POINTER(C.c_double)),
                ("naux", C.c_int), ("aux", C.c_void_p), ("src", C.c_void_p), ("bdata", C.c_void_p),
                ("nbc", C.c_int), ("bc_kind", C.POINTER(C.c_int32))]


class GmresOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("maxit", C.c_int), ("flexible", C.c_int), ("rtol", C.c_double),
                ("atol", C.c_double), ("jvp_prec", C.c_int), ("pc", C.c_void_p), ("inject_fault", C.c_int),
                ("orth", C.c_int), ("state32", C.c_int), ("watch_window", C.c_int),
                ("record_v", C.c_void_p), ("record_jz", C.c_void_p), ("record_max", C.c_int)]


class GmresStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("fell_back", C.c_int), ("res0", C.c_double),
                ("res_est", C.c_double), ("res_true", C.c_double), ("t_jvp", C.c_double), ("t_pc", C.c_double),
                ("t_orth", C.c_double), ("t_total", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NewtonOpts(C.Structure):
    _fields_ = [("maxit", C.c_int), ("rtol", C.c_double), ("atol", C.c_double), ("eta", C.c_double),
                ("bj_refresh", C.c_int), ("bj_per_variable", C.c_int), ("bj_prec", C.c_int), ("lin", GmresOpts)]


class NewtonStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("gmres_iters", C.c_int), ("res0", C.c_double), ("res_final", C.c_double),
                ("seconds", C.c_double), ("lin_status", C.c_int), ("t_jvp", C.c_double), ("t_pc", C.c_double),
                ("t_orth", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

EXPORTED = ["ldg_last_error", "ldg_mesh_create", "ldg_mesh_info", "ldg_mesh_points", "ldg_mesh_destroy",
            "ldg_model_create", "ldg_model_destroy", "ldg_residual", "ldg_jvp", "ldg_jvp_prepare", "ldg_jvp_prepared",
            "ldg_jvp_state32",
            "ldg_jacobian_blocks",
            "ldg_precond_block_jacobi", "ldg_precond_apply", "ldg_precond_destroy", "ldg_gmres_solve",
            "ldg_newton_solve", "ldg_axpby", "ldg_norm2", "ldg_mlp_create", "ldg_mlp_destroy", "ldg_mlp_set_params",
            "ldg_mlp_get_params", "ldg_mlp_forward", "ldg_mlp_forward_noalloc", "ldg_mlp_train_step",
            "ldg_mlp_train_step_bilinear", "ldg_mlp_gather_patches",
            "ldg_precond_mlp", "ldg_model_create_user", "ldg_user_physics_check", "ldg_ode_size", "ldg_ode_stage"]


def lib():
    """Load libldg.so; fails loudly if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    vp, dp, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)
    L.ldg_last_error.restype = C.c_char_p
    sig = {
        "ldg_mesh_create": [C.c_int, C.c_int, C.c_int, C.c_int64, dp, C.c_int64, i64p, dp, C.POINTER(C.c_int32),
                            C.POINTER(vp)],
        "ldg_mesh_info": [vp, i64p],
        "ldg_mesh_points": [vp, dp, dp, dp, i64p],
        "ldg_mesh_destroy": [vp],
        "ldg_model_create": [vp, C.POINTER(_ModelDesc), vp, C.POINTER(vp)],
        "ldg_model_destroy": [vp],
        "ldg_residual": [vp, C.POINTER(_Time), vp, vp, vp, C.c_int, vp],
        "ldg_jvp": [vp, C.POINTER(_Time), vp, vp, vp, C.c_int, vp],
        "ldg_jvp_prepare": [vp, vp, C.c_int, vp],
        "ldg_jvp_state32": [vp, C.POINTER(_Time), vp, vp, vp, vp],
        "ldg_jvp_prepared": [vp, C.POINTER(_Time), vp, vp, vp, C.c_int, vp],
        "ldg_jacobian_blocks": [vp, C.POINTER(_Time), vp, C.c_int, vp, vp],
        "ldg_precond_block_jacobi": [vp, C.POINTER(_Time), vp, C.c_int, C.c_int, vp, C.POINTER(vp)],
        "ldg_precond_apply": [vp, vp, vp, vp],
        "ldg_precond_destroy": [vp],
        "ldg_gmres_solve": [vp, C.POINTER(_Time), vp, vp, vp, C.POINTER(GmresOpts), C.POINTER(GmresStats), vp],
        "ldg_newton_solve": [vp, C.POINTER(_Time), vp, C.POINTER(NewtonOpts), C.POINTER(NewtonStats), vp],
        "ldg_axpby": [C.c_int64, C.c_double, vp, C.c_double, vp, vp],
        "ldg_norm2": [C.c_int64, vp, dp, vp],
        "ldg_mlp_create": [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(vp)],
        "ldg_mlp_destroy": [vp],
        "ldg_mlp_set_params": [vp, C.POINTER(C.c_float)],
        "ldg_mlp_get_params": [vp, C.POINTER(C.c_float), C.POINTER(C.c_float)],
        "ldg_mlp_forward": [vp, vp, C.c_int64, vp, vp],
        "ldg_mlp_forward_noalloc": [vp, vp, C.c_int64, vp, vp],
        "ldg_mlp_train_step": [vp, vp, vp, C.c_int64, C.c_float, C.POINTER(C.c_float), vp],
        "ldg_mlp_train_step_bilinear": [vp, vp, vp, C.c_int64, C.c_float, C.POINTER(C.c_float), vp],
        "ldg_mlp_gather_patches": [vp, vp, vp, vp, C.c_int64, vp, vp, vp, vp],
        "ldg_precond_mlp": [vp, vp, vp, C.c_int, C.POINTER(vp)],
        "ldg_model_create_user": [vp, C.POINTER(_ModelDesc), C.c_char_p, C.c_int, vp, C.POINTER(vp)],
        "ldg_user_physics_check": [C.c_char_p, C.c_int, C.c_int, C.c_int, C.c_int],
        "ldg_ode_size": [vp, C.POINTER(C.c_int)],
        "ldg_ode_stage": [vp, C.POINTER(_Time), C.c_double, C.c_double, vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    _lib = L
    return L


def _check(status, what=""):
    if status != LDG_OK:
        raise LDGError(status, f"{what}: {lib().ldg_last_error().decode()}")


def _ptr(t, what="tensor", dtype=torch.float64, numel=None, optional=True):
    """Device pointer of a tensor after checking what the C ABI assumes of it: a contiguous
    HIP tensor of the given dtype and element count.  Any mismatch raises ValueError here,
    before a wrong-sized or wrong-typed buffer can reach a kernel."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{what}: required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{what}: must be a device (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what}: dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: {t.numel()} elements, expected {numel}")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ----------------------------------------------------------------------------
class Mesh:
    def __init__(self, box, p, nq=None):
        self.nd, self.p = box.nd, p
        self.nq = p + 1 if nq is None else nq
        v = _np(box.vert, np.float64)
        ev = _np(box.elem_vert, np.int64)
        per = _np(box.period, np.float64)
        ft = _np(box.face_tag, np.int32)
        h = C.c_void_p()
        _check(lib().ldg_mesh_create(self.nd, p, self.nq, v.shape[0], v.ctypes.data_as(C.POINTER(C.c_double)),
                                     ev.shape[0], ev.ctypes.data_as(C.POINTER(C.c_int64)),
                                     per.ctypes.data_as(C.POINTER(C.c_double)),
                                     ft.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(h)), "ldg_mesh_create")
        self.h = h
        info = np.zeros(8, dtype=np.int64)
        _check(lib().ldg_mesh_info(h, info.ctypes.data_as(C.POINTER(C.c_int64))), "ldg_mesh_info")
        self.E, self.nn, self.nqv, self.nqf, self.nbf, self.ncolors, self.affine, _ = (int(x) for x in info)

    def points(self):
        xn = np.zeros((self.E, self.nn, self.nd))
        xq = np.zeros((self.E, self.nqv, self.nd))
        xb = np.zeros((max(self.nbf, 1), self.nqf, self.nd))
        bf = np.zeros((max(self.nbf, 1), 2), dtype=np.int64)
        dp = C.POINTER(C.c_double)
        _check(lib().ldg_mesh_points(self.h, xn.ctypes.data_as(dp), xq.ctypes.data_as(dp), xb.ctypes.data_as(dp),
                                     bf.ctypes.data_as(C.POINTER(C.c_int64))), "ldg_mesh_points")
        return xn, xq, xb[:self.nbf], bf[:self.nbf]

    def size(self, ncu):
        return self.E * ncu * self.nn

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ldg_mesh_destroy(self.h)
            self.h = None


@dataclass
class Time:
    """G(u) = a0 M u - M (c1 r1 + c2 r2) + R(u)."""
    a0: float = 0.0
    r1: torch.Tensor = None
    c1: float = 0.0
    r2: torch.Tensor = None
    c2: float = 0.0

    def c(self, n):
        """ABI struct; r1 and r2 must be FP64 device vectors of n entries (any length when n is None: the call
        reads neither, e.g. an ODE stage of a model without an ODE, which the library rejects)."""
        self._c = _Time(self.a0, _ptr(self.r1, "time.r1", numel=n), self.c1, _ptr(self.r2, "time.r2", numel=n),
                        self.c2)
        return C.byref(self._c)


def _time(t, n):
    return None if t is None else t.c(n)


class Model:
    """A model bound to a mesh.  kind = MODEL_USER takes physics_source (the LdgUser struct, compiled at run time
    by the library) and has_q."""

    def __init__(self, mesh, kind, ncu, mu, aux=None, src=None, bdata=None, bc_kind=(0,), physics_source=None,
                 has_q=True):
        self.mesh, self.kind, self.ncu = mesh, kind, ncu
        dev = torch.device("cuda")
        def to(a):
            if a is None:
                return None
            if isinstance(a, torch.Tensor):
                return a.to(device=dev, dtype=torch.float64).contiguous()
            return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).to(dev).contiguous()
        # keep the device copies alive for the lifetime of the model
        self.aux, self.src, self.bdata = to(aux), to(src), to(bdata)
        self._mu = _np(mu, np.float64)
        self._bc = _np(bc_kind, np.int32)
        naux = 0 if self.aux is None else int(self.aux.numel() // max(mesh.E * mesh.nn, 1))
        E, nn = mesh.E, mesh.nn
        d = _ModelDesc(kind, ncu, len(self._mu), self._mu.ctypes.data_as(C.POINTER(C.c_double)), naux,
                       _ptr(self.aux, "aux [E][naux][nn]", numel=E * naux * nn),
                       _ptr(self.src, "src [E][ncu][nqv]", numel=E * ncu * mesh.nqv),
                       _ptr(self.bdata, "bdata [nbf][ncu][nqf]", numel=mesh.nbf * ncu * mesh.nqf), len(self._bc),
                       self._bc.ctypes.data_as(C.POINTER(C.c_int32)))
        h = C.c_void_p()
        if physics_source is not None:
            _check(lib().ldg_model_create_user(mesh.h, C.byref(d), physics_source.encode(), int(has_q), _stream(),
                                               C.byref(h)), "ldg_model_create_user")
        else:
            _check(lib().ldg_model_create(mesh.h, C.byref(d), _stream(), C.byref(h)), "ldg_model_create")
        self.h = h
        self.N = mesh.size(ncu)
        nw = C.c_int()
        _check(lib().ldg_ode_size(h, C.byref(nw)), "ldg_ode_size")
        self.nw = nw.value          # components of the coupled ODE (Eq. 1c); 0 without one

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ldg_model_destroy(self.h)
            self.h = None

    def empty(self):
        return torch.empty(self.N, dtype=torch.float64, device="cuda")

    def residual(self, u, time=None, prec=FP64, q_out=None, out=None):
        out = self.empty() if out is None else out
        N = self.N
        _check(lib().ldg_residual(self.h, _time(time, N), _ptr(u, "u", numel=N, optional=False),
                                  _ptr(out, "out", numel=N), _ptr(q_out, "q_out", numel=N * self.mesh.nd), prec,
                                  _stream()), "ldg_residual")
        return out

    def jvp(self, u, v, time=None, prec=FP64, out=None):
        out = self.empty() if out is None else out
        N = self.N
        _check(lib().ldg_jvp(self.h, _time(time, N), _ptr(u, "u", numel=N), _ptr(v, "v", numel=N, optional=False),
                             _ptr(out, "out", numel=N), prec, _stream()), "ldg_jvp")
        return out

    def jvp_prepare(self, u, prec=FP64):
        """Cache q(u) in the model for jvp_prepared (the solvers' linearization point)."""
        _check(lib().ldg_jvp_prepare(self.h, _ptr(u, "u", numel=self.N, optional=False), prec, _stream()),
               "ldg_jvp_prepare")

    def jvp_prepared(self, u, v, time=None, prec=FP64, out=None):
        """J(u) v with q(u) from the last jvp_prepare(u, prec)."""
        out = self.empty() if out is None else out
        N = self.N
        _check(lib().ldg_jvp_prepared(self.h, _time(time, N), _ptr(u, "u", numel=N),
                                      _ptr(v, "v", numel=N, optional=False), _ptr(out, "out", numel=N), prec,
                                      _stream()), "ldg_jvp_prepared")
        return out

    def jvp_state32(self, u, v, time=None, out=None):
        """J(u) v with u and v in FP32 storage (FP32 arithmetic), Jv in FP64."""
        out = self.empty() if out is None else out
        N = self.N
        f32 = torch.float32
        _check(lib().ldg_jvp_state32(self.h, _time(time, N), _ptr(u, "u [FP32]", f32, N),
                                     _ptr(v, "v [FP32]", f32, N, optional=False), _ptr(out, "out", numel=N),
                                     _stream()), "ldg_jvp_state32")
        return out

    def ode_stage(self, u, time, alpha, beta, out=None):
        """w of one implicit stage of alpha dw/dt + beta w = s_w(u) with the time wrapper `time` (its r1, r2 are
        w-vectors), from the stage's PDE state u."""
        nwv = self.mesh.E * self.nw * self.mesh.nn
        out = torch.empty(max(nwv, 1), dtype=torch.float64, device="cuda") if out is None else out
        if time is None:
            raise ValueError("ode_stage: a time wrapper is required")
        # without an ODE (nw = 0) the library returns LDG_EUNSUPPORTED before it reads any vector
        nchk = nwv if self.nw > 0 else None
        _check(lib().ldg_ode_stage(self.h, _time(time, nchk), C.c_double(alpha), C.c_double(beta),
                                   _ptr(u, "u", numel=self.N, optional=False), _ptr(out, "out", numel=nchk),
                                   _stream()), "ldg_ode_stage")
        return out

    def jacobian_blocks(self, u, time=None, per_variable=False):
        nn = self.mesh.nn
        if per_variable:
            out = torch.zeros((self.mesh.E, self.ncu, nn, nn), dtype=torch.float64, device="cuda")
        else:
            nb = self.ncu * nn
            out = torch.zeros((self.mesh.E, nb, nb), dtype=torch.float64, device="cuda")
        _check(lib().ldg_jacobian_blocks(self.h, _time(time, self.N), _ptr(u, "u", numel=self.N), int(per_variable),
                                         _ptr(out), _stream()), "ldg_jacobian_blocks")
        return out


class BlockJacobi:
    def __init__(self, model, u_lin=None, time=None, per_variable=False, prec=FP64):
        self.model = model
        h = C.c_void_p()
        _check(lib().ldg_precond_block_jacobi(model.h, _time(time, model.N), _ptr(u_lin, "u_lin", numel=model.N),
                                              int(per_variable), prec, _stream(), C.byref(h)),
               "ldg_precond_block_jacobi")
        self.h = h

    def apply(self, r, out=None):
        out = self.model.empty() if out is None else out
        N = self.model.N
        _check(lib().ldg_precond_apply(self.h, _ptr(r, "r", numel=N, optional=False), _ptr(out, "out", numel=N),
                                       _stream()), "ldg_precond_apply")
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ldg_precond_destroy(self.h)
            self.h = None


class MLP:
    """3-layer element-patch network; params packed W1 b1 W2 b2 W3 b3 (row-major W[out][in])."""

    def __init__(self, in_dim, width, out_dim, bf16=True):
        self.dims = (in_dim, width, out_dim)
        h = C.c_void_p()
        _check(lib().ldg_mlp_create(in_dim, width, out_dim, 3, int(bf16), C.byref(h)), "ldg_mlp_create")
        self.h = h
        self.shapes = [(width, in_dim), (width,), (width, width), (width,), (out_dim, width), (out_dim,)]
        self.nparams = int(sum(np.prod(s) for s in self.shapes))

    def set_params(self, params):
        flat = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.float32).reshape(-1) for p in params]))
        assert flat.size == self.nparams
        _check(lib().ldg_mlp_set_params(self.h, flat.ctypes.data_as(C.POINTER(C.c_float))), "ldg_mlp_set_params")

    def _unpack(self, flat):
        out, o = [], 0
        for s in self.shapes:
            n = int(np.prod(s))
            out.append(flat[o:o + n].reshape(s).copy())
            o += n
        return out

    def get_params(self):
        p = np.zeros(self.nparams, dtype=np.float32)
        g = np.zeros(self.nparams, dtype=np.float32)
        _check(lib().ldg_mlp_get_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)),
                                        g.ctypes.data_as(C.POINTER(C.c_float))), "ldg_mlp_get_params")
        return self._unpack(p), self._unpack(g)

    def forward(self, X, out=None):
        B = X.shape[0]
        out = torch.empty((B, self.dims[2]), dtype=torch.float32, device="cuda") if out is None else out
        f32 = torch.float32
        _check(lib().ldg_mlp_forward(self.h, _ptr(X, "X [B][in]", f32, B * self.dims[0], optional=False), B,
                                     _ptr(out, "out [B][out]", f32, B * self.dims[2], optional=False), _stream()),
               "ldg_mlp_forward")
        return out

    def forward_noalloc(self, X, out):
        """ldg_mlp_forward_noalloc: the forward pass with the library's fixed scratch array (no device allocation
        in the call); out [B][out] must be given."""
        B = X.shape[0]
        f32 = torch.float32
        _check(lib().ldg_mlp_forward_noalloc(self.h, _ptr(X, "X [B][in]", f32, B * self.dims[0], optional=False), B,
                                             _ptr(out, "out [B][out]", f32, B * self.dims[2], optional=False),
                                             _stream()), "ldg_mlp_forward_noalloc")
        return out

    def train_step(self, X, Y, lr):
        loss = C.c_float()
        B = X.shape[0]
        f32 = torch.float32
        _check(lib().ldg_mlp_train_step(self.h, _ptr(X, "X [B][in]", f32, B * self.dims[0], optional=False),
                                        _ptr(Y, "Y [B][out]", f32, B * self.dims[2], optional=False), B, float(lr),
                                        C.byref(loss), _stream()), "ldg_mlp_train_step")
        return float(loss.value)

    def train_step_bilinear(self, X, Y, lr):
        """ldg_mlp_train_step_bilinear: X [B][20 nn] patch features (residual patch, then the coefficient
        features the network reads), Y [B][nn] targets of A_b r_b."""
        loss = C.c_float()
        B = X.shape[0]
        f32 = torch.float32
        nn = self.dims[0] // 15
        _check(lib().ldg_mlp_train_step_bilinear(self.h, _ptr(X, "X [B][20 nn]", f32, B * 20 * nn, optional=False),
                                                 _ptr(Y, "Y [B][nn]", f32, B * nn, optional=False), B, float(lr),
                                                 C.byref(loss), _stream()), "ldg_mlp_train_step_bilinear")
        return float(loss.value)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ldg_mlp_destroy(self.h)
            self.h = None


def gather_patches(model, r, e=None, elems=None, want_scale=False):
    B = model.mesh.E if elems is None else elems.numel()
    nn = model.mesh.nn
    if elems is not None and B > 0:
        lo, hi = int(elems.min()), int(elems.max())
        if lo < 0 or hi >= model.mesh.E:
            raise ValueError(f"elems: indices must lie in [0, {model.mesh.E}), got [{lo}, {hi}]")
    X = torch.empty((B, 20 * nn), dtype=torch.float32, device="cuda")
    Y = torch.empty((B, nn), dtype=torch.float32, device="cuda") if e is not None else None
    S = torch.empty(B, dtype=torch.float64, device="cuda") if want_scale else None
    N = model.N
    _check(lib().ldg_mlp_gather_patches(model.h, _ptr(r, "r", numel=N, optional=False), _ptr(e, "e", numel=N),
                                        _ptr(elems, "elems", torch.int32), B, _ptr(X, dtype=torch.float32),
                                        _ptr(Y, dtype=torch.float32), _ptr(S), _stream()),
           "ldg_mlp_gather_patches")
    return X, Y, S


class LearnedPrecond:
    """ldg_precond_mlp.  composite: False / 0 (network alone), True / 1 (block-Jacobi + network correction of
    the residual form) or "linear" / 2 (z = B^-1 (r + A_K patch(r)), A_K from the coefficient patch)."""

    def __init__(self, model, net, bj, composite=True):
        self.model, self.net, self.bj = model, net, bj
        form = 2 if composite == "linear" else int(composite)
        h = C.c_void_p()
        _check(lib().ldg_precond_mlp(model.h, net.h, None if bj is None else bj.h, form, C.byref(h)),
               "ldg_precond_mlp")
        self.h = h

    def apply(self, r, out=None):
        out = self.model.empty() if out is None else out
        N = self.model.N
        _check(lib().ldg_precond_apply(self.h, _ptr(r, "r", numel=N, optional=False), _ptr(out, "out", numel=N),
                                       _stream()), "ldg_precond_apply")
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ldg_precond_destroy(self.h)
            self.h = None


ORTH_CGS2, ORTH_MGS, ORTH_DCGS2 = 0, 1, 2


def gmres_opts(restart=30, maxit=1000, rtol=1e-8, atol=0.0, jvp_prec=FP64, pc=None, flexible=True, inject_fault=0,
               orth=ORTH_DCGS2, state32=False, watch_window=0, record=None):
    """record = (V, JZ): two contiguous FP64 device tensors [k][N] that receive, for the first k steps of the
    solve, the preconditioner's input v_i and the product J z_i of its output (ldg_gmres_opts.record_*)."""
    rz = rj = None
    rmax = 0
    if record is not None:
        V, JZ = record
        if V.shape != JZ.shape or V.dim() != 2:
            raise ValueError("record: two tensors of equal shape [k][N]")
        rz, rj = _ptr(V, "record V", optional=False), _ptr(JZ, "record JZ", optional=False)
        rmax = V.shape[0]
    return GmresOpts(restart, maxit, int(flexible), rtol, atol, jvp_prec, None if pc is None else pc.h, inject_fault,
                     orth, int(state32), int(watch_window), rz, rj, rmax)


def gmres(model, b, x=None, u_lin=None, time=None, check=True, **kw):
    x = torch.zeros_like(b) if x is None else x
    N = model.N
    rec = kw.get("record")
    if rec is not None and any(t.dim() != 2 or t.shape[1] != N for t in rec):
        raise ValueError(f"record: tensors [k][{N}] expected")
    o = gmres_opts(**kw)
    st = GmresStats()
    status = lib().ldg_gmres_solve(model.h, _time(time, N), _ptr(u_lin, "u_lin", numel=N),
                                   _ptr(b, "b", numel=N, optional=False), _ptr(x, "x", numel=N, optional=False),
                                   C.byref(o), C.byref(st), _stream())
    if check and status not in (LDG_OK,):
        _check(status, "ldg_gmres_solve")
    return x, st.as_dict(), status


def newton(model, u, time=None, maxit=20, rtol=1e-8, atol=0.0, eta=1e-3, bj_refresh=False, bj_per_variable=False,
           bj_prec=FP64, check=True, lin_maxit=1000, **lin):
    o = NewtonOpts(maxit, rtol, atol, eta, int(bj_refresh), int(bj_per_variable), bj_prec,
                   gmres_opts(maxit=lin_maxit, **lin))
    st = NewtonStats()
    status = lib().ldg_newton_solve(model.h, _time(time, model.N), _ptr(u, "u", numel=model.N, optional=False),
                                    C.byref(o), C.byref(st), _stream())
    if check and status != LDG_OK:
        _check(status, "ldg_newton_solve")
    return u, st.as_dict(), status


def user_physics_check(source, nd, p, ncu, has_q=True):
    """Compile a physics source on the host only (no device); raises LDGError with the compiler's log."""
    _check(lib().ldg_user_physics_check(source.encode(), nd, p, ncu, int(has_q)), "ldg_user_physics_check")


def axpby(a, x, b, y):
    """y = a x + b y on the device (FP64 vectors of equal length)."""
    n = x.numel()
    _check(lib().ldg_axpby(n, C.c_double(a), _ptr(x, "x", optional=False), C.c_double(b),
                           _ptr(y, "y", numel=n, optional=False), _stream()), "ldg_axpby")
    return y


def norm(x):
    out = C.c_double()
    _check(lib().ldg_norm2(x.numel(), _ptr(x, "x", optional=False), C.byref(out), _stream()), "ldg_norm2")
    return float(np.sqrt(out.value))
