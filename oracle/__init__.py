"""CPU oracle for the LDG residual / Jacobian path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library: the discrete
operator lives in ``ldg_oracle.cpp`` (plain FP64 C++, built with g++), and the
solvers below (FGMRES with modified Gram-Schmidt and Givens rotations, Newton,
the learned-preconditioner MLP) are plain numpy written from their textbook
definitions.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ldg_oracle.cpp")
_LIB = os.path.join(_HERE, "libldg_oracle.so")

MODEL_POISSON, MODEL_CONVDIFF, MODEL_EULER, MODEL_NS, MODEL_SHALLOW_WATER, MODEL_WAVE = 0, 1, 2, 3, 4, 5
BC_DIRICHLET, BC_NEUMANN, BC_EXTRAP, BC_SLIP_WALL = 0, 1, 2, 3


def build(force=True):
    """Compile the oracle with g++ (-O2, no fast-math, single thread)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip64 = C.POINTER(C.c_int64)
        L.ldgo_last_error.restype = C.c_char_p
        L.ldgo_lagrange.restype = C.c_double
        L.ldgo_lagrange.argtypes = [C.c_int, dp, C.c_int, C.c_double, C.c_int]
        L.ldgo_mesh_create.restype = C.c_void_p
        L.ldgo_mesh_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int64, dp, C.c_int64, ip64, dp,
                                       C.POINTER(C.c_int32)]
        L.ldgo_mesh_destroy.argtypes = [C.c_void_p]
        L.ldgo_mesh_info.argtypes = [C.c_void_p, ip64]
        L.ldgo_mesh_points.argtypes = [C.c_void_p, dp, dp, dp, ip64]
        L.ldgo_mesh_geometry_checks.argtypes = [C.c_void_p, dp, dp]
        L.ldgo_mesh_neighbours.argtypes = [C.c_void_p, ip64]
        L.ldgo_residual.argtypes = [C.c_void_p, C.c_void_p, dp, dp, dp]
        L.ldgo_jvp.argtypes = [C.c_void_p, C.c_void_p, dp, dp, dp, dp]
        L.ldgo_jacobian_coo.restype = C.c_int64
        L.ldgo_jacobian_coo.argtypes = [C.c_void_p, C.c_void_p, dp, C.c_int64, ip64, ip64, dp]
        L.ldgo_jacobian_blocks.argtypes = [C.c_void_p, C.c_void_p, dp, C.c_int64, ip64, C.c_int, dp]
        L.ldgo_sample_elements.argtypes = [C.c_void_p, C.c_void_p, dp, dp, C.c_int64, ip64, dp, dp]
        L.ldgo_mass_apply.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.ldgo_lu_factor.argtypes = [C.c_int, dp, C.POINTER(C.c_int)]
        L.ldgo_lu_solve.argtypes = [C.c_int, dp, C.POINTER(C.c_int), dp]
        L.ldgo_error_points.argtypes = [C.c_void_p, C.c_int, dp]
        L.ldgo_l2_error.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, dp]
        L.ldgo_point_flux.argtypes = [C.c_void_p, C.c_int, dp, dp, dp, dp]
        L.ldgo_point_numflux.argtypes = [C.c_void_p, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.ldgo_set_tie_break.restype = C.c_int
        L.ldgo_set_tie_break.argtypes = [C.c_int]
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i64(a):
    if a is None:
        return None
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _err():
    return lib().ldgo_last_error().decode()


class _ModelDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("ncu", C.c_int), ("nmu", C.c_int), ("mu", C.POINTER(C.c_double)),
                ("naux", C.c_int), ("aux", C.POINTER(C.c_double)), ("src", C.POINTER(C.c_double)),
                ("bdata", C.POINTER(C.c_double)), ("nbc", C.c_int), ("bc_kind", C.POINTER(C.c_int)),
                ("a0", C.c_double), ("r", C.POINTER(C.c_double))]


class Model:
    """Model description: kind, parameters, coefficient fields and boundary data.

    aux   [E][naux][nn]   nodal coefficient fields (kappa factor; kappa and b)
    src   [E][ncu][nqv]   source sampled at the volume quadrature points
    bdata [nbf][ncu][nqf] boundary data at boundary-face quadrature points
    a0, r                 time wrapper G = a0 M u - M r + R(u)
    """

    def __init__(self, kind, ncu, mu, aux=None, src=None, bdata=None, bc_kind=(0,), a0=0.0, r=None, naux=0):
        self.kind, self.ncu = kind, ncu
        self.mu = np.ascontiguousarray(mu, dtype=np.float64)
        self.aux = None if aux is None else np.ascontiguousarray(aux, dtype=np.float64)
        self.naux = naux if aux is None else self.aux.shape[1]
        self.src = None if src is None else np.ascontiguousarray(src, dtype=np.float64)
        self.bdata = None if bdata is None else np.ascontiguousarray(bdata, dtype=np.float64)
        self.bc_kind = np.ascontiguousarray(bc_kind, dtype=np.int32)
        self.a0 = float(a0)
        self.r = None if r is None else np.ascontiguousarray(r, dtype=np.float64)

    def replace(self, **kw):
        d = dict(kind=self.kind, ncu=self.ncu, mu=self.mu, aux=self.aux, src=self.src, bdata=self.bdata,
                 bc_kind=self.bc_kind, a0=self.a0, r=self.r)
        d.update(kw)
        return Model(**d)

    def desc(self):
        self._desc = _ModelDesc(self.kind, self.ncu, len(self.mu), _d(self.mu), self.naux, _d(self.aux),
                                _d(self.src), _d(self.bdata), len(self.bc_kind),
                                self.bc_kind.ctypes.data_as(C.POINTER(C.c_int)), self.a0, _d(self.r))
        return C.byref(self._desc)


class Mesh:
    """Oracle mesh: Gauss-Legendre nodal basis of degree p, nq quadrature points per direction."""

    def __init__(self, box, p, nq=None):
        self.nd, self.p = box.nd, p
        self.nq = p + 1 if nq is None else nq
        self._keep = (np.ascontiguousarray(box.vert, dtype=np.float64),
                      np.ascontiguousarray(box.elem_vert, dtype=np.int64),
                      np.ascontiguousarray(box.period, dtype=np.float64),
                      np.ascontiguousarray(box.face_tag, dtype=np.int32))
        v, ev, per, ft = self._keep
        self.h = lib().ldgo_mesh_create(self.nd, p, self.nq, v.shape[0], _d(v), ev.shape[0], _i64(ev), _d(per),
                                        ft.ctypes.data_as(C.POINTER(C.c_int32)))
        if not self.h:
            raise RuntimeError("oracle mesh: " + _err())
        info = np.zeros(5, dtype=np.int64)
        lib().ldgo_mesh_info(self.h, _i64(info))
        self.E, self.nn, self.nqv, self.nqf, self.nbf = (int(x) for x in info)

    def __del__(self):
        if getattr(self, "h", None):
            lib().ldgo_mesh_destroy(self.h)
            self.h = None

    def points(self):
        xn = np.zeros((self.E, self.nn, self.nd))
        xq = np.zeros((self.E, self.nqv, self.nd))
        xb = np.zeros((max(self.nbf, 1), self.nqf, self.nd))
        bf = np.zeros((max(self.nbf, 1), 2), dtype=np.int64)
        lib().ldgo_mesh_points(self.h, _d(xn), _d(xq), _d(xb), _i64(bf))
        return xn, xq, xb[:self.nbf], bf[:self.nbf]

    def geometry_checks(self):
        vol = np.zeros(self.E)
        ns = np.zeros((self.E, self.nd))
        lib().ldgo_mesh_geometry_checks(self.h, _d(vol), _d(ns))
        return vol, ns

    def neighbours(self):
        nb = np.zeros((self.E, 2 * self.nd), dtype=np.int64)
        lib().ldgo_mesh_neighbours(self.h, _i64(nb))
        return nb

    def size(self, ncu):
        return self.E * ncu * self.nn

    # ---- operator ------------------------------------------------------------
    def residual(self, model, u, want_q=False):
        u = np.ascontiguousarray(u, dtype=np.float64)
        R = np.zeros(self.size(model.ncu))
        q = np.zeros(self.E * model.ncu * self.nd * self.nn) if want_q else None
        if lib().ldgo_residual(self.h, model.desc(), _d(u), _d(R), _d(q)) != 0:
            raise RuntimeError("oracle residual: " + _err())
        return (R, q) if want_q else R

    def jvp(self, model, u, v, want_dq=False):
        u = np.ascontiguousarray(u, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        Jv = np.zeros(self.size(model.ncu))
        dq = np.zeros(self.E * model.ncu * self.nd * self.nn) if want_dq else None
        if lib().ldgo_jvp(self.h, model.desc(), _d(u), _d(v), _d(Jv), _d(dq)) != 0:
            raise RuntimeError("oracle jvp: " + _err())
        return (Jv, dq) if want_dq else Jv

    def jacobian(self, model, u):
        """Sparse Jacobian dG/du (scipy CSR) assembled column by column."""
        import scipy.sparse as sp
        u = np.ascontiguousarray(u, dtype=np.float64)
        N = self.size(model.ncu)
        nb = model.ncu * self.nn
        cap = N * nb * (1 + 2 * self.nd + 2 * self.nd * self.nd) + 16
        rows = np.zeros(cap, dtype=np.int64)
        cols = np.zeros(cap, dtype=np.int64)
        vals = np.zeros(cap)
        nnz = lib().ldgo_jacobian_coo(self.h, model.desc(), _d(u), cap, _i64(rows), _i64(cols), _d(vals))
        if nnz < 0:
            raise RuntimeError("oracle jacobian: " + _err())
        return sp.csr_matrix((vals[:nnz], (rows[:nnz], cols[:nnz])), shape=(N, N))

    def blocks(self, model, u, elems=None, per_variable=False):
        u = np.ascontiguousarray(u, dtype=np.float64)
        elems = np.arange(self.E, dtype=np.int64) if elems is None else np.ascontiguousarray(elems, dtype=np.int64)
        nb = model.ncu * self.nn
        if per_variable:
            out = np.zeros((len(elems), model.ncu, self.nn, self.nn))
        else:
            out = np.zeros((len(elems), nb, nb))
        if lib().ldgo_jacobian_blocks(self.h, model.desc(), _d(u), len(elems), _i64(elems), int(per_variable),
                                      _d(out)) != 0:
            raise RuntimeError("oracle blocks: " + _err())
        return out

    def sample(self, model, u, v, elems):
        """G_K(u) and (J(u) v)_K on the listed elements: [len(elems)][ncu*nn] each."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        v = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
        elems = np.ascontiguousarray(elems, dtype=np.int64)
        nb = model.ncu * self.nn
        G = np.zeros((len(elems), nb))
        Jv = np.zeros((len(elems), nb))
        if lib().ldgo_sample_elements(self.h, model.desc(), _d(u), _d(v), len(elems), _i64(elems), _d(G),
                                      _d(Jv)) != 0:
            raise RuntimeError("oracle sample: " + _err())
        return G, Jv

    def mass_apply(self, ncu, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        out = np.zeros_like(u)
        lib().ldgo_mass_apply(self.h, ncu, _d(u), _d(out))
        return out

    def error_points(self, m):
        x = np.zeros((self.E, m ** self.nd, self.nd))
        lib().ldgo_error_points(self.h, m, _d(x))
        return x

    def l2_error(self, m, ncu, c, u, q, uex, qex):
        out = np.zeros(4)
        u = np.ascontiguousarray(u, dtype=np.float64)
        q = None if q is None else np.ascontiguousarray(q, dtype=np.float64)
        lib().ldgo_l2_error(self.h, m, ncu, c, _d(u), _d(q), _d(np.ascontiguousarray(uex, dtype=np.float64)),
                            _d(None if qex is None else np.ascontiguousarray(qex, dtype=np.float64)), _d(out))
        return out[0] / out[1], (out[2] / out[3] if q is not None else None)


class tie_break:
    """Context manager selecting the one-sided derivative the dual numbers take at an
    exact kink: +1 is the default convention (sign(0) = +1, a max tie takes the first
    argument's tangent), -1 the other side."""

    def __init__(self, t):
        self.t = t

    def __enter__(self):
        self.old = lib().ldgo_set_tie_break(int(self.t))
        return self

    def __exit__(self, *exc):
        lib().ldgo_set_tie_break(self.old)
        return False


def gauss_legendre(m):
    x = np.zeros(m)
    w = np.zeros(m)
    lib().ldgo_gauss_legendre(m, _d(x), _d(w))
    return x, w


def lagrange(nodes, i, x, deriv=False):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    return lib().ldgo_lagrange(len(nodes), _d(nodes), i, float(x), int(deriv))


def point_flux(model, nd, u, q, a):
    f = np.zeros(model.ncu * nd)
    lib().ldgo_point_flux(model.desc(), nd, _d(np.ascontiguousarray(u, float)), _d(np.ascontiguousarray(q, float)),
                          _d(np.ascontiguousarray(a, float)), _d(f))
    return f.reshape(model.ncu, nd)


def point_numflux(model, nd, uL, qL, aL, uR, qR, aR, n):
    F = np.zeros(model.ncu)
    a = [np.ascontiguousarray(t, float) for t in (uL, qL, aL, uR, qR, aR, n)]
    lib().ldgo_point_numflux(model.desc(), nd, *[_d(t) for t in a], _d(F))
    return F


# ----------------------------------------------------------------------------
# Block LU (Doolittle, partial pivoting) of the element blocks
# ----------------------------------------------------------------------------
class BlockLU:
    def __init__(self, blocks):
        self.B = np.ascontiguousarray(blocks, dtype=np.float64).copy()
        nblk, n, _ = self.B.shape
        self.piv = np.zeros((nblk, n), dtype=np.int32)
        for b in range(nblk):
            blk = self.B[b]
            pv = self.piv[b]
            if lib().ldgo_lu_factor(n, blk.ctypes.data_as(C.POINTER(C.c_double)),
                                    pv.ctypes.data_as(C.POINTER(C.c_int))) != 0:
                raise RuntimeError("singular block")

    def solve(self, r):
        nblk, n, _ = self.B.shape
        z = np.ascontiguousarray(r, dtype=np.float64).reshape(nblk, n).copy()
        for b in range(nblk):
            zb = z[b]
            lib().ldgo_lu_solve(n, self.B[b].ctypes.data_as(C.POINTER(C.c_double)),
                                self.piv[b].ctypes.data_as(C.POINTER(C.c_int)), zb.ctypes.data_as(C.POINTER(C.c_double)))
        return z.reshape(-1)


# ----------------------------------------------------------------------------
# O10: flexible GMRES(m), right preconditioning, modified Gram-Schmidt, Givens
# (Saad & Schultz 1986; Saad 1993 for the flexible variant)
# ----------------------------------------------------------------------------
def fgmres(A, b, x0=None, M=None, restart=30, maxit=1000, rtol=1e-10, atol=0.0, history=None):
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.astype(np.float64).copy()
    M = (lambda v: v) if M is None else M
    r = b - A(x)
    r0 = np.linalg.norm(r)
    tol = max(rtol * r0, atol)
    its = 0
    beta = r0
    info = dict(iters=0, restarts=0, res0=r0, converged=beta <= tol)
    while its < maxit and beta > tol:
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            Z[j] = M(V[j])
            w = A(Z[j])
            wnorm0 = np.linalg.norm(w)
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] <= 1e-14 * wnorm0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            if history is not None:
                history.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= tol or breakdown or its >= maxit:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + Z[:k].T @ y
        r = b - A(x)
        beta = np.linalg.norm(r)
        info["restarts"] += 1
    info["iters"] = its
    info["res_true"] = beta
    info["converged"] = beta <= tol * (1 + 1e-6) or beta <= tol + 1e-300
    return x, info


# ----------------------------------------------------------------------------
# O11: Newton's method with a linear solver callback
# ----------------------------------------------------------------------------
def newton(G, solve, u0, rtol=1e-8, atol=0.0, maxit=20, history=None):
    u = u0.astype(np.float64).copy()
    g = G(u)
    g0 = np.linalg.norm(g)
    hist = [g0] if history is None else history
    if history is not None:
        history.append(g0)
    k = 0
    while k < maxit and np.linalg.norm(g) > max(rtol * g0, atol):
        du = solve(u, -g)
        u = u + du
        g = G(u)
        hist.append(np.linalg.norm(g))
        k += 1
    return u, dict(iters=k, res0=g0, res=np.linalg.norm(g))


# ----------------------------------------------------------------------------
# O11b: diagonally implicit Runge-Kutta time stepping of M du/dt + R(u) = 0
# (Section 2: the paper's DIRK discretization in time, schemes after Alexander
# 1977).  Written from the stage equations themselves:
#   M (U_i - u_n) / dt + sum_{j<=i} a_ij R(U_j) = 0,   i = 1..s,
#   u_{n+1} = u_n + dt sum_j b_j k_j,   k_j = -M^{-1} R(U_j),
# each stage solved by Newton with sparse direct solves of
# M/dt + a_ii dR/du.  M is diagonal for the collocated nodal basis.
# ----------------------------------------------------------------------------
def dirk_tableau(name):
    """(A, b) of implicit Euler ("be"), Alexander's L-stable two- and three-stage schemes of orders 2 and 3
    ("dirk22", "dirk33", with b the last row of A) and the three-stage fourth-order A-stable scheme ("dirk34")."""
    if name == "be":
        return np.array([[1.0]]), np.array([1.0])
    if name == "dirk22":
        g = (2.0 - np.sqrt(2.0)) / 2.0
        return np.array([[g, 0.0], [1.0 - g, g]]), np.array([1.0 - g, g])
    if name == "dirk33":
        roots = np.roots([1.0, -3.0, 1.5, -1.0 / 6.0])
        g = float(next(r.real for r in roots if abs(r.imag) < 1e-12 and 1.0 / 6.0 < r.real < 0.5))
        t2 = (1.0 + g) / 2.0
        b1 = -(6.0 * g ** 2 - 16.0 * g + 1.0) / 4.0
        b2 = (6.0 * g ** 2 - 20.0 * g + 5.0) / 4.0
        A = np.array([[g, 0.0, 0.0], [t2 - g, g, 0.0], [b1, b2, g]])
        return A, A[2].copy()
    if name == "dirk34":
        g = 0.5 + np.cos(np.pi / 18.0) / np.sqrt(3.0)
        d = 1.0 / (6.0 * (2.0 * g - 1.0) ** 2)
        return (np.array([[g, 0.0, 0.0], [0.5 - g, g, 0.0], [2.0 * g, 1.0 - 4.0 * g, g]]),
                np.array([d, 1.0 - 2.0 * d, d]))
    raise ValueError(name)


def dirk_step(mesh, model, un, dt, A, b, rtol=1e-13, maxit=12, ode=None):
    """One DIRK step of M du/dt + R(u) = 0 from un; model is the steady model (its R).  Returns u_{n+1}.

    ode = (s_w, alpha, beta, w_n): the ODE coupled to the PDE (Eq. 1c), alpha dw/dt + beta w = s_w(u), with
    s_w a function of the nodal state vector.  It runs through the same Butcher stages: W_i = w_n +
    dt sum_j a_ij Wdot_j with alpha Wdot_i + beta W_i = s_w(U_i), so Wdot_i = (s_w(U_i) - beta (w_n +
    dt sum_{j<i} a_ij Wdot_j)) / (alpha + beta dt a_ii); then w_{n+1} = w_n + dt sum_j b_j Wdot_j.
    With ode the result is (u_{n+1}, w_{n+1})."""
    import scipy.sparse.linalg as spla
    ncu = model.ncu
    Mdiag = mesh.mass_apply(ncu, np.ones_like(un))
    s = len(b)
    R = []
    Wdot = []
    U = un.copy()
    for i in range(s):
        rest = sum((A[i, j] * R[j] for j in range(i)), np.zeros_like(un))

        def F(x, i=i, rest=rest):
            return mesh.mass_apply(ncu, x - un) / dt + rest + A[i, i] * mesh.residual(model, x)

        # dF/du = M/dt + a_ii dR/du = a_ii (a0 M + dR/du) with a0 = 1/(a_ii dt)
        mj = model.replace(a0=1.0 / (A[i, i] * dt), r=None)

        def solve(x, rhs, i=i, mj=mj):
            return spla.spsolve((A[i, i] * mesh.jacobian(mj, x)).tocsc(), rhs)

        U, info = newton(F, solve, U, rtol=rtol, maxit=maxit)
        R.append(mesh.residual(model, U))
        if ode is not None:
            s_w, alpha, beta, wn = ode
            base = wn + dt * sum((A[i, j] * Wdot[j] for j in range(i)), np.zeros_like(wn))
            Wdot.append((s_w(U) - beta * base) / (alpha + beta * dt * A[i, i]))
    k = [-Rj / Mdiag for Rj in R]
    u_next = un + dt * sum(b[j] * k[j] for j in range(s))
    if ode is None:
        return u_next
    return u_next, ode[3] + dt * sum(b[j] * Wdot[j] for j in range(s))


# ----------------------------------------------------------------------------
# O12: the element-patch MLP in FP64: y = W3 relu(W2 relu(W1 x + b1) + b2) + b3,
# hand-written backward pass and Adam.
# ----------------------------------------------------------------------------
def mlp_forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3.T + b3
    return y, (X, z1, h1, z2, h2)


def mlp_loss_and_grad(params, X, Y):
    """Mean squared error 1/(B*out) sum (y - Y)^2 and its gradient w.r.t. the parameters."""
    y, cache = mlp_forward(params, X)
    B, nout = Y.shape
    diff = y - Y
    loss = np.sum(diff * diff) / (B * nout)
    return loss, _mlp_backward(params, cache, 2.0 * diff / (B * nout))


def mlp_bilinear_loss_and_grad(params, X, Y, nn):
    """The linear form's loss.  Row b of X holds the residual patch r_b = X[b, :5 nn]
    and the coefficient features c_b = X[b, 5 nn:]; the network maps c_b to the
    row-major matrix A_b [nn][5 nn] and predicts A_b r_b.  Loss 1/(B nn) sum
    (A_b r_b - Y_b)^2; by the chain rule its gradient with respect to A_b is
    dy_b r_b^T, which the network's backward pass takes from there."""
    R, Cf = X[:, :5 * nn], X[:, 5 * nn:]
    out, cache = mlp_forward(params, Cf)
    B = X.shape[0]
    A = out.reshape(B, nn, 5 * nn)
    y = np.einsum("bij,bj->bi", A, R)
    diff = y - Y
    loss = np.sum(diff * diff) / (B * nn)
    dy = 2.0 * diff / (B * nn)
    dout = (dy[:, :, None] * R[:, None, :]).reshape(B, nn * 5 * nn)
    return loss, _mlp_backward(params, cache, dout)


def linear_patch_precond(Binv, A, nbrs, r):
    """The linear form of the learned preconditioner, z = B^-1 (r + A_K patch(r)_K)
    per element K: Binv [E][nn][nn] the inverse diagonal blocks, A [E][nn][5 nn],
    nbrs [E][4] the face neighbours (-x, +x, -y, +y; -1 outside, where the patch
    holds zeros)."""
    E, nn = Binv.shape[0], Binv.shape[1]
    R = r.reshape(E, nn)
    z = np.zeros((E, nn))
    for K in range(E):
        patch = np.concatenate([R[k] if k >= 0 else np.zeros(nn) for k in [K] + [int(x) for x in nbrs[K]]])
        z[K] = Binv[K] @ (R[K] + A[K] @ patch)
    return z.reshape(-1)


def _mlp_backward(params, cache, dy):
    """Parameter gradients of the network from the gradient dy of the loss with respect to its output."""
    W1, b1, W2, b2, W3, b3 = params
    X, z1, h1, z2, h2 = cache
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dh2 = dy @ W3
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    out = []
    for i, (p, g) in enumerate(zip(params, grads)):
        m[i] = b1 * m[i] + (1 - b1) * g
        v[i] = b2 * v[i] + (1 - b2) * g * g
        mh = m[i] / (1 - b1 ** t)
        vh = v[i] / (1 - b2 ** t)
        out.append(p - lr * mh / (np.sqrt(vh) + eps))
    return out
