"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the LDG method: it only builds meshes
(vertex coordinates + connectivity), analytic fields (manufactured solutions,
initial states, random coefficient fields) and random vectors.  Both the
HIP library and the CPU oracle consume what it returns; each side computes its
own quadrature points, geometry and operators.

Workload shapes follow the configurations the method is exercised on:

* 2D Poisson, 8x8 unit square, manufactured sin(pi x) sin(pi y);
* 3D Poisson/heat, 32^3 unit cube, interior vertices perturbed by +-5% of h,
  manufactured exp(x+y+z) sin(pi x y z);
* 2D Euler, periodic [0,20]^2, superposed isentropic vortices;
* 3D Navier-Stokes Taylor-Green vortex on the periodic (0,2 pi)^3 box;
* shallow-water Bickley jet on the periodic (-2 pi, 2 pi)^2 box;
* 2D convection-diffusion with a log-normal random kappa and a
  divergence-free velocity.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# ----------------------------------------------------------------------------
# Box meshes
# ----------------------------------------------------------------------------
@dataclass
class BoxMesh:
    nd: int
    n: tuple            # elements per direction
    lo: tuple
    hi: tuple
    periodic: tuple
    vert: np.ndarray       # [nvert][nd] float64
    elem_vert: np.ndarray  # [E][2^nd] int64, corners lexicographic (bit k <-> +side in dir k)
    period: np.ndarray     # [nd] float64, 0 = not periodic
    face_tag: np.ndarray   # [E][2nd] int32: 2k+s on boundary faces, -1 on interior faces

    @property
    def nelem(self):
        return self.elem_vert.shape[0]

    @property
    def h(self):
        return tuple((self.hi[k] - self.lo[k]) / self.n[k] for k in range(self.nd))


def box_mesh(nd, n, lo=None, hi=None, periodic=None, perturb=0.0, seed=0):
    """Structured quad/hex mesh of a box.

    n: int or tuple of elements per direction.  Periodic directions reuse the
    vertex plane at the low end for the high end (vertices are identified, so
    the connectivity wraps).  ``perturb`` moves every vertex that is not on the
    box boundary by U(-perturb*h, perturb*h) per coordinate (numpy
    default_rng(seed)); boundary vertices stay fixed so the domain is unchanged.
    """
    if isinstance(n, int):
        n = (n,) * nd
    lo = tuple(lo) if lo is not None else (0.0,) * nd
    hi = tuple(hi) if hi is not None else (1.0,) * nd
    periodic = tuple(periodic) if periodic is not None else (False,) * nd
    nvd = [n[k] if periodic[k] else n[k] + 1 for k in range(nd)]
    h = [(hi[k] - lo[k]) / n[k] for k in range(nd)]
    # vertex lattice, x fastest
    grids = np.meshgrid(*[lo[k] + h[k] * np.arange(nvd[k]) for k in range(nd)], indexing="ij")
    vert = np.stack([g.transpose(tuple(range(nd))[::-1]).reshape(-1) for g in grids], axis=1)
    # the transpose above makes the flattened order x-fastest
    vert = np.ascontiguousarray(vert, dtype=np.float64)
    if perturb > 0.0:
        rng = np.random.default_rng(seed)
        idx = np.indices(nvd[::-1]).reshape(nd, -1)[::-1]  # idx[k] = lattice index in dir k
        interior = np.ones(vert.shape[0], dtype=bool)
        for k in range(nd):
            if not periodic[k]:
                interior &= (idx[k] > 0) & (idx[k] < n[k])
        disp = rng.uniform(-1.0, 1.0, size=vert.shape) * (perturb * np.asarray(h))[None, :]
        vert = vert + disp * interior[:, None]

    strides = [1] * nd
    for k in range(1, nd):
        strides[k] = strides[k - 1] * nvd[k - 1]
    eidx = np.indices(n[::-1]).reshape(nd, -1)[::-1]  # element lattice indices, x fastest
    E = eidx.shape[1]
    nv = 1 << nd
    elem_vert = np.zeros((E, nv), dtype=np.int64)
    for c in range(nv):
        vid = np.zeros(E, dtype=np.int64)
        for k in range(nd):
            ik = eidx[k] + ((c >> k) & 1)
            if periodic[k]:
                ik = ik % n[k]
            vid += ik * strides[k]
        elem_vert[:, c] = vid
    face_tag = -np.ones((E, 2 * nd), dtype=np.int32)
    for k in range(nd):
        if periodic[k]:
            continue
        face_tag[eidx[k] == 0, 2 * k] = 2 * k
        face_tag[eidx[k] == n[k] - 1, 2 * k + 1] = 2 * k + 1
    period = np.array([(hi[k] - lo[k]) if periodic[k] else 0.0 for k in range(nd)])
    return BoxMesh(nd, tuple(n), lo, hi, periodic, vert, elem_vert, period, face_tag)


# ----------------------------------------------------------------------------
# Manufactured solutions (exact fields and their sources for -lap u = f)
# ----------------------------------------------------------------------------
def mms_sin2d(x):
    """u = sin(pi x) sin(pi y); returns (u, grad u [.., 2], f = -lap u)."""
    X, Y = x[..., 0], x[..., 1]
    u = np.sin(np.pi * X) * np.sin(np.pi * Y)
    g = np.stack([np.pi * np.cos(np.pi * X) * np.sin(np.pi * Y),
                  np.pi * np.sin(np.pi * X) * np.cos(np.pi * Y)], axis=-1)
    return u, g, 2.0 * np.pi ** 2 * u


def mms_sin3d(x):
    """u = sin(pi x) sin(pi y) sin(pi z)."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    sx, sy, sz = np.sin(np.pi * X), np.sin(np.pi * Y), np.sin(np.pi * Z)
    cx, cy, cz = np.cos(np.pi * X), np.cos(np.pi * Y), np.cos(np.pi * Z)
    u = sx * sy * sz
    g = np.pi * np.stack([cx * sy * sz, sx * cy * sz, sx * sy * cz], axis=-1)
    return u, g, 3.0 * np.pi ** 2 * u


def mms_expsin3d(x):
    """u = exp(x+y+z) sin(pi x y z) with f = -lap u in closed form."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    eg = np.exp(X + Y + Z)
    S = np.sin(np.pi * X * Y * Z)
    C = np.cos(np.pi * X * Y * Z)
    u = eg * S
    g = np.stack([eg * (S + np.pi * Y * Z * C),
                  eg * (S + np.pi * X * Z * C),
                  eg * (S + np.pi * X * Y * C)], axis=-1)
    lap = eg * (3.0 * S + 2.0 * np.pi * C * (X * Y + Y * Z + Z * X)
                - np.pi ** 2 * S * (X * X * Y * Y + Y * Y * Z * Z + Z * Z * X * X))
    return u, g, -lap


def mms_poly(x, coeffs, degs):
    """Sum of monomials c * prod x_k^{e_k}; returns (u, grad u, -lap u)."""
    nd = x.shape[-1]
    u = np.zeros(x.shape[:-1])
    g = np.zeros(x.shape)
    lap = np.zeros(x.shape[:-1])
    for c, e in zip(coeffs, degs):
        mono = c * np.prod([x[..., k] ** e[k] for k in range(nd)], axis=0)
        u += mono
        for k in range(nd):
            if e[k] >= 1:
                t = c * e[k] * np.prod([x[..., j] ** (e[j] - (1 if j == k else 0)) for j in range(nd)], axis=0)
                g[..., k] += t
            if e[k] >= 2:
                t = c * e[k] * (e[k] - 1) * np.prod(
                    [x[..., j] ** (e[j] - (2 if j == k else 0)) for j in range(nd)], axis=0)
                lap += t
    return u, g, -lap


# ----------------------------------------------------------------------------
# Euler / Navier-Stokes initial states (conservative variables)
# ----------------------------------------------------------------------------
def vortex_centres(n, L, min_sep, seed):
    rng = np.random.default_rng(seed)
    cs = []
    while len(cs) < n:
        c = rng.uniform(0.0, L, size=2)
        ok = True
        for d in cs:
            dd = np.abs(c - d)
            dd = np.minimum(dd, L - dd)
            if math.hypot(*dd) < min_sep:
                ok = False
                break
        if ok:
            cs.append(c)
    return np.array(cs)


def isentropic_vortices(x, centres, L=20.0, gamma=1.4, beta=5.0, mach=0.5):
    """Superposed isentropic vortices on a uniform stream along +x.

    Free stream rho=p=T=1, speed mach*sqrt(gamma).  Each vortex adds the
    classical velocity and temperature perturbations; distances use the
    minimum periodic image.  Returns [.., 4] = (rho, rho u, rho v, rho E)."""
    X, Y = x[..., 0], x[..., 1]
    vinf = mach * math.sqrt(gamma)
    du = np.zeros(X.shape)
    dv = np.zeros(X.shape)
    dT = np.zeros(X.shape)
    for c in centres:
        xb = X - c[0]
        yb = Y - c[1]
        xb = xb - L * np.round(xb / L)
        yb = yb - L * np.round(yb / L)
        r2 = xb * xb + yb * yb
        e = np.exp(0.5 * (1.0 - r2))
        du += -beta / (2 * np.pi) * e * yb
        dv += beta / (2 * np.pi) * e * xb
        dT += -(gamma - 1.0) * beta ** 2 / (8.0 * gamma * np.pi ** 2) * e * e
    T = 1.0 + dT
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    vx = vinf + du
    vy = dv
    E = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy)
    return np.stack([rho, rho * vx, rho * vy, E], axis=-1)


def bickley_jet(x, seed=0, eps=0.01, nmodes=4, L=4.0 * math.pi):
    """Shallow-water Bickley jet on the periodic box (-L/2, L/2)^2 (the paper's second convection workload).

    Depth h = 1 and velocity u = sech^2(y), v = 0, plus a slight seeded
    perturbation of the velocity: eps times a sum of nmodes x-periodic modes
    (wavenumbers 1..nmodes in units of 2 pi / L, random phases and amplitudes)
    localized on the jet by exp(-y^2).  Returns [.., 3] = (h, h u, h v)."""
    X, Y = x[..., 0], x[..., 1]
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2.0 * np.pi, (2, nmodes))
    amp = rng.uniform(0.5, 1.0, (2, nmodes))
    env = np.exp(-Y * Y)
    du = np.zeros(X.shape)
    dv = np.zeros(X.shape)
    for k in range(nmodes):
        w = 2.0 * np.pi * (k + 1) / L
        du += amp[0, k] * np.cos(w * X + ph[0, k])
        dv += amp[1, k] * np.sin(w * X + ph[1, k])
    h = np.ones(X.shape)
    vx = 1.0 / np.cosh(Y) ** 2 + eps * env * du
    vy = eps * env * dv
    return np.stack([h, h * vx, h * vy], axis=-1)


def taylor_green(x, gamma=1.4, mach=0.1):
    """Taylor-Green vortex on (0, 2 pi)^3, isothermal density.  [.., 5]."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    p0 = 1.0 / (gamma * mach * mach)
    p = p0 + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    rho = p / p0
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E], axis=-1)


# ----------------------------------------------------------------------------
# Convection-diffusion coefficient fields
# ----------------------------------------------------------------------------
@dataclass
class GRF:
    """log-normal field via random Fourier features: log k = sqrt(2/M) sum cos(w.x + b).

    w ~ N(0, ell^-2 I), b ~ U(0, 2 pi): zero mean, unit variance and
    squared-exponential covariance exp(-r^2 / (2 ell^2))."""
    omega: np.ndarray
    phase: np.ndarray

    @staticmethod
    def sample(seed, ell=0.1, M=1024, nd=2):
        rng = np.random.default_rng(seed)
        return GRF(rng.normal(0.0, 1.0 / ell, size=(M, nd)), rng.uniform(0.0, 2 * np.pi, size=M))

    def log_kappa(self, x):
        M = self.phase.shape[0]
        arg = x.reshape(-1, x.shape[-1]) @ self.omega.T + self.phase[None, :]
        return (math.sqrt(2.0 / M) * np.cos(arg).sum(axis=1)).reshape(x.shape[:-1])

    def log_kappa_on(self, x, device, chunk=65536):
        """The same sum evaluated with torch in FP64 on a device (a torch tensor of
        shape x.shape[:-1]); it agrees with log_kappa to rounding and serves sweeps
        over many instances, where the host evaluation would dominate."""
        import torch
        M = self.phase.shape[0]
        pts = torch.as_tensor(np.ascontiguousarray(x.reshape(-1, x.shape[-1])), dtype=torch.float64, device=device)
        om = torch.as_tensor(self.omega, dtype=torch.float64, device=device)
        ph = torch.as_tensor(self.phase, dtype=torch.float64, device=device)
        out = torch.empty(pts.shape[0], dtype=torch.float64, device=device)
        for s in range(0, pts.shape[0], chunk):
            out[s:s + chunk] = torch.cos(pts[s:s + chunk] @ om.T + ph).sum(dim=1)
        return (out * math.sqrt(2.0 / M)).reshape(x.shape[:-1])


@dataclass
class DivFreeVelocity:
    """b = A * perp-grad(psi) / max|perp-grad(psi)|, psi a sum of 8 Fourier modes."""
    k: np.ndarray
    amp: np.ndarray
    ph: np.ndarray
    A: float
    scale: float

    @staticmethod
    def sample(seed, nmodes=8, kmax=4, Amin=1.0, Amax=100.0):
        rng = np.random.default_rng(seed + 7919)
        k = 2 * np.pi * rng.integers(1, kmax + 1, size=(nmodes, 2)).astype(np.float64)
        k *= rng.choice([-1.0, 1.0], size=(nmodes, 2))
        amp = rng.normal(size=nmodes)
        ph = rng.uniform(0, 2 * np.pi, size=nmodes)
        A = float(np.exp(rng.uniform(np.log(Amin), np.log(Amax))))
        obj = DivFreeVelocity(k, amp, ph, A, 1.0)
        g = np.stack(np.meshgrid(np.linspace(0, 1, 257), np.linspace(0, 1, 257), indexing="ij"), -1)
        obj.scale = float(np.max(np.linalg.norm(obj._perp_grad(g), axis=-1)))
        return obj

    def _perp_grad(self, x):
        arg = x @ self.k.T + self.ph
        c = np.cos(arg) * self.amp
        dpsi_dx = (c * self.k[:, 0]).sum(-1)
        dpsi_dy = (c * self.k[:, 1]).sum(-1)
        return np.stack([dpsi_dy, -dpsi_dx], axis=-1)

    def __call__(self, x):
        return self.A * self._perp_grad(x) / self.scale


def random_vector(n, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=n)
