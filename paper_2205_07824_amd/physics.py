"""Pointwise physics sources of the paper's other models, for ldg_model_create_user.

The library compiles such a source at run time with the operator kernels
(Section 3: code generated from the PDE's description).  SHALLOW_WATER_2D is
the shallow-water system (h, h v) with the local Lax-Friedrichs flux (speed
|v.n| + sqrt(g h)), the paper's Bickley-jet model (Section 4).  WAVE_2D is the
paper's wave model written as a first-order system in (u, q) with the upwind
(Lax-Friedrichs, speed c) flux; WAVE_2D_W adds the coupled ODE (Eq. 1c) for the
displacement, w_t = u.  EULER_2D re-states the compressible Euler flux and the
local Lax-Friedrichs flux in the same format (a compiled model comparable with
the built-in Euler model); EULER_2D_SLIP adds slip walls through a boundary
function.  NONLINEAR_DIFFUSION is a model the library has no kernel for:
f = kappa q with kappa = mu0 kappa(x) (1 + mu2 u^2) (kappa(x) an optional aux
field), central flux plus an interior penalty mu1 mu0 {kappa(x)} (u- - u+);
with mu2 = 0 it is the built-in Poisson operator without reaction.  REACTION_DIFFUSION
adds a state-dependent source s(u) (Eq. 1b), REACTION_DIFFUSION_BOU also a
boundary function on one tag.
"""

EULER_2D = r"""
struct LdgUser {
  static constexpr int NCU = 4;
  static constexpr bool HASQ = false;
  static constexpr int NAUX = 0;
  template <int D, class V, class R>
  __device__ static void flux(const double* mu, int, const V* u, const V (*)[D], const R*, V (*f)[D]) {
    const R gam = R(mu[0]);
    const V rho = u[0], E = u[D + 1];
    const V rinv = VT<V>::mk(R(1)) / rho;
    V vel[D];
    V ke = VT<V>::mk(R(0));
    for (int k = 0; k < D; ++k) { vel[k] = u[1 + k] * rinv; ke += u[1 + k] * vel[k]; }
    const V p = (gam - R(1)) * (E - R(0.5) * ke);
    for (int k = 0; k < D; ++k) {
      f[0][k] = u[1 + k];
      for (int i = 0; i < D; ++i) {
        f[1 + i][k] = u[1 + i] * vel[k];
        if (i == k) f[1 + i][k] += p;
      }
      f[D + 1][k] = (E + p) * vel[k];
    }
  }
  template <int D, class V, class R>
  __device__ static V speed(R gam, const V* u, const R* n) {
    const V rinv = VT<V>::mk(R(1)) / u[0];
    V vn = VT<V>::mk(R(0)), ke = VT<V>::mk(R(0));
    for (int k = 0; k < D; ++k) { vn += (u[1 + k] * rinv) * n[k]; ke += u[1 + k] * u[1 + k] * rinv; }
    const V p = (gam - R(1)) * (u[D + 1] - R(0.5) * ke);
    return vabs(vn) + vsqrt(gam * p * rinv);
  }
  template <int D, class V, class R>
  __device__ static void numflux(const double* mu, int naux, const V* uL, const V (*qL)[D], const R* aL,
                                 const V* uR, const V (*qR)[D], const R* aR, const R* n, V* Fh) {
    V f[NCU][D];
    flux<D, V, R>(mu, naux, uL, qL, aL, f);
    for (int c = 0; c < NCU; ++c) {
      V s = f[c][0] * n[0];
      for (int k = 1; k < D; ++k) s += f[c][k] * n[k];
      Fh[c] = R(0.5) * s;
    }
    flux<D, V, R>(mu, naux, uR, qR, aR, f);
    for (int c = 0; c < NCU; ++c) {
      V s = f[c][0] * n[0];
      for (int k = 1; k < D; ++k) s += f[c][k] * n[k];
      Fh[c] += R(0.5) * s;
    }
    const V sig = R(0.5) * vmax(speed<D, V, R>(R(mu[0]), uL, n), speed<D, V, R>(R(mu[0]), uR, n));
    for (int c = 0; c < NCU; ++c) Fh[c] += sig * (uL[c] - uR[c]);
  }
};
"""

NONLINEAR_DIFFUSION = r"""
struct LdgUser {
  static constexpr int NCU = 1;
  static constexpr bool HASQ = true;
  static constexpr int NAUX = 1;   // optional kappa(x) field
  template <int D, class V, class R>
  __device__ static void flux(const double* mu, int naux, const V* u, const V (*q)[D], const R* a, V (*f)[D]) {
    const R kx = naux >= 1 ? a[0] : R(1);
    const V kap = (R(mu[0]) * kx) * (VT<V>::mk(R(1)) + R(mu[2]) * u[0] * u[0]);
    for (int k = 0; k < D; ++k) f[0][k] = kap * q[0][k];
  }
  template <int D, class V, class R>
  __device__ static void numflux(const double* mu, int naux, const V* uL, const V (*qL)[D], const R* aL,
                                 const V* uR, const V (*qR)[D], const R* aR, const R* n, V* Fh) {
    V fL[1][D], fR[1][D];
    flux<D, V, R>(mu, naux, uL, qL, aL, fL);
    flux<D, V, R>(mu, naux, uR, qR, aR, fR);
    V s = R(0.5) * (fL[0][0] + fR[0][0]) * n[0];
    for (int k = 1; k < D; ++k) s += R(0.5) * (fL[0][k] + fR[0][k]) * n[k];
    const R kbar = naux >= 1 ? R(0.5) * (aL[0] + aR[0]) : R(1);
    Fh[0] = s + (R(mu[1]) * R(mu[0]) * kbar) * (uL[0] - uR[0]);
  }
};
"""

SHALLOW_WATER_2D = r"""
struct LdgUser {
  static constexpr int NCU = 3;
  static constexpr bool HASQ = false;
  static constexpr int NAUX = 0;
  // u = (h, h v); g = mu[0]
  template <int D, class V, class R>
  __device__ static void flux(const double* mu, int, const V* u, const V (*)[D], const R*, V (*f)[D]) {
    const V hinv = VT<V>::mk(R(1)) / u[0];
    const V pg = R(0.5 * mu[0]) * u[0] * u[0];
    for (int k = 0; k < D; ++k) {
      f[0][k] = u[1 + k];
      const V vk = u[1 + k] * hinv;
      for (int i = 0; i < D; ++i) f[1 + i][k] = u[1 + i] * vk + (i == k ? pg : VT<V>::mk(R(0)));
    }
  }
  template <int D, class V, class R>
  __device__ static V speed(R g, const V* u, const R* n) {
    const V hinv = VT<V>::mk(R(1)) / u[0];
    V vn = VT<V>::mk(R(0));
    for (int k = 0; k < D; ++k) vn += (u[1 + k] * hinv) * n[k];
    return vabs(vn) + vsqrt(g * u[0]);
  }
  template <int D, class V, class R>
  __device__ static void numflux(const double* mu, int naux, const V* uL, const V (*qL)[D], const R* aL,
                                 const V* uR, const V (*qR)[D], const R* aR, const R* n, V* Fh) {
    V fL[NCU][D], fR[NCU][D];
    flux<D, V, R>(mu, naux, uL, qL, aL, fL);
    flux<D, V, R>(mu, naux, uR, qR, aR, fR);
    const V sig = R(0.5) * vmax(speed<D, V, R>(R(mu[0]), uL, n), speed<D, V, R>(R(mu[0]), uR, n));
    for (int c = 0; c < NCU; ++c) {
      V s = R(0.5) * (fL[c][0] + fR[c][0]) * n[0];
      for (int k = 1; k < D; ++k) s += R(0.5) * (fL[c][k] + fR[c][k]) * n[k];
      Fh[c] = s + sig * (uL[c] - uR[c]);
    }
  }
};
"""

WAVE_2D = r"""
struct LdgUser {
  static constexpr int NCU = 3;      // state (u, q1, q2)
  static constexpr bool HASQ = false;
  static constexpr int NAUX = 0;
  // u_t + div(c^2 q) = 0, q_t + grad u = 0: f = (c^2 q, u I), c^2 = mu[0]
  template <int D, class V, class R>
  __device__ static void flux(const double* mu, int, const V* u, const V (*)[D], const R*, V (*f)[D]) {
    for (int k = 0; k < D; ++k) {
      f[0][k] = R(mu[0]) * u[1 + k];
      for (int i = 0; i < D; ++i) f[1 + i][k] = (i == k) ? u[0] : VT<V>::mk(R(0));
    }
  }
  template <int D, class V, class R>
  __device__ static void numflux(const double* mu, int naux, const V* uL, const V (*qL)[D], const R* aL,
                                 const V* uR, const V (*qR)[D], const R* aR, const R* n, V* Fh) {
    V fL[NCU][D], fR[NCU][D];
    flux<D, V, R>(mu, naux, uL, qL, aL, fL);
    flux<D, V, R>(mu, naux, uR, qR, aR, fR);
    const R sig = R(0.5) * R(sqrt(mu[0]));
    for (int c = 0; c < NCU; ++c) {
      V s = R(0.5) * (fL[c][0] + fR[c][0]) * n[0];
      for (int k = 1; k < D; ++k) s += R(0.5) * (fL[c][k] + fR[c][k]) * n[k];
      Fh[c] = s + sig * (uL[c] - uR[c]);
    }
  }
};
"""

# Euler with slip walls on tags 2 and 3 (the outside state reverses the normal momentum) and the boundary
# data elsewhere
EULER_2D_SLIP = EULER_2D.replace("static constexpr int NAUX = 0;", """static constexpr int NAUX = 0;
  static constexpr bool BOU = true;
  template <int D, class V, class R>
  __device__ static void bou(const double*, int, int tag, const V* uL, const V (*)[D], const R*, const R* n,
                             V* ub) {
    if (tag != 2 && tag != 3) return;
    V mn = uL[1] * n[0];
    for (int k = 1; k < D; ++k) mn += uL[1 + k] * n[k];
    for (int c = 0; c < NCU; ++c) ub[c] = uL[c];
    for (int k = 0; k < D; ++k) ub[1 + k] = uL[1 + k] - R(2) * mn * n[k];
  }""", 1)

# the wave model with the paper's displacement ODE (w_t = u, first component) and a second, nonlinear
# component s_w = mu[1] q1 q2, so that a sum of two fields and a product are both checked
WAVE_2D_W = WAVE_2D.replace("static constexpr int NAUX = 0;", """static constexpr int NAUX = 0;
  static constexpr int NW = 2;
  __device__ static void ode_source(const double* mu, int, const double* u, const double*, double* sw) {
    sw[0] = u[0];
    sw[1] = mu[1] * u[1] * u[2];
  }""", 1)

# NONLINEAR_DIFFUSION with the state-dependent source s(u) = -(mu3 u + mu4 u^3) of Eq. 1b (a reaction term):
# at mu2 = mu4 = 0 it is the built-in Poisson model with reaction lambda = mu3
REACTION_DIFFUSION = NONLINEAR_DIFFUSION.replace("static constexpr int NAUX = 1;   // optional kappa(x) field", """static constexpr int NAUX = 1;   // optional kappa(x) field
  static constexpr bool SOURCE = true;
  template <int D, class V, class R>
  __device__ static void source(const double* mu, int, const V* u, const V (*)[D], const R*, V* s) {
    s[0] = -(R(mu[3]) * u[0] + R(mu[4]) * (u[0] * u[0]) * u[0]);
  }""", 1)

# REACTION_DIFFUSION with a boundary function on tag 1: the outside state of the numerical flux is
# g + mu5 uL^2 (the gradient's boundary trace stays the data g, the outside gradient q+ = q-)
REACTION_DIFFUSION_BOU = REACTION_DIFFUSION.replace("static constexpr bool SOURCE = true;", """static constexpr bool SOURCE = true;
  static constexpr bool BOU = true;
  template <int D, class V, class R>
  __device__ static void bou(const double* mu, int, int tag, const V* uL, const V (*)[D], const R*, const R*,
                             V* ub) {
    if (tag == 1) ub[0] = ub[0] + R(mu[5]) * uL[0] * uL[0];
  }""", 1)
