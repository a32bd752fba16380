// Pointwise physics of the built-in models: flux f(u, q) [NCU][D], numerical
// flux across a face, max wave speed.  Written once for plain values and for
// dual numbers (value, tangent), so that the tangent kernels differentiate
// exactly the arithmetic of the residual kernels.
#pragma once

#include "ldg_device.hpp"

namespace ldg {

enum { K_POISSON = 0, K_CONVDIFF = 1, K_EULER = 2, K_NS = 3, K_USER = 4 };

template <int KIND, int D>
struct Phys {
  static constexpr int NCU = (KIND <= 1) ? 1 : D + 2;
  static constexpr bool HASQ = (KIND != K_EULER);
  static constexpr bool LINEAR = (KIND <= 1);
  static constexpr int NAUX = (KIND == K_CONVDIFF) ? 1 + D : (KIND == K_POISSON ? 1 : 0);
};

// User physics (a model compiled at run time): the source defines a struct
// LdgUser with NCU, HASQ, NAUX and the templates flux<D>(mu, naux, u, q, a, f)
// and numflux<D>(mu, naux, uL, qL, aL, uR, qR, aR, n, Fh), written once for
// plain values and dual numbers like the built-in models below.
#ifdef LDG_USER_PHYSICS
template <int D>
struct Phys<K_USER, D> {
  static constexpr int NCU = ::LdgUser::NCU;
  static constexpr bool HASQ = ::LdgUser::HASQ;
  static constexpr bool LINEAR = false;
  static constexpr int NAUX = ::LdgUser::NAUX;
};
#endif

// physical flux; a = aux at the point (R), naux = number of aux fields present
template <int KIND, int D, class V, class R>
__device__ inline void phys_flux(const double* mu, int naux, const V* u, const V (*q)[D], const R* a,
                                 V (*f)[D]) {
  using T = VT<V>;
  if constexpr (KIND == K_POISSON) {
    R kap = R(mu[0]) * (naux >= 1 ? a[0] : R(1));
#pragma unroll
    for (int k = 0; k < D; ++k) f[0][k] = kap * q[0][k];
  }
#ifdef LDG_USER_PHYSICS
  else if constexpr (KIND == K_USER) {
    ::LdgUser::template flux<D, V, R>(mu, naux, u, q, a, f);
  }
#endif
  else if constexpr (KIND == K_CONVDIFF) {
    R kap = R(mu[0]) * a[0];
#pragma unroll
    for (int k = 0; k < D; ++k) f[0][k] = kap * q[0][k] + a[1 + k] * u[0];
  } else {
    const R gam = R(mu[0]);
    constexpr int NE = D + 1;
    V rho = u[0], E = u[NE];
    V rinv = T::mk(R(1)) / rho;
    V vel[D];
    V ke = T::mk(R(0));
#pragma unroll
    for (int k = 0; k < D; ++k) { vel[k] = u[1 + k] * rinv; ke += u[1 + k] * vel[k]; }
    V pr = (gam - R(1)) * (E - R(0.5) * ke);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      f[0][k] = u[1 + k];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        f[1 + i][k] = u[1 + i] * vel[k];
        if (i == k) f[1 + i][k] += pr;
      }
      f[NE][k] = (E + pr) * vel[k];
    }
    if constexpr (KIND == K_NS) {
      const R vis = R(1) / R(mu[1]);
      const R kcond = vis * gam / R(mu[2]);
      V gv[D][D], ge[D];
      V Em = E * rinv;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        V gr = -q[0][k];                     // grad u = -q
#pragma unroll
        for (int i = 0; i < D; ++i) gv[i][k] = (-q[1 + i][k] - vel[i] * gr) * rinv;
        V gEm = (-q[NE][k] - Em * gr) * rinv;
        V s = gEm;
#pragma unroll
        for (int i = 0; i < D; ++i) s -= vel[i] * gv[i][k];
        ge[k] = s;
      }
      V divv = gv[0][0];
#pragma unroll
      for (int i = 1; i < D; ++i) divv += gv[i][i];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        V work = T::mk(R(0));
#pragma unroll
        for (int i = 0; i < D; ++i) {
          V tau = vis * (gv[i][k] + gv[k][i]);
          if (i == k) tau -= (vis * R(2.0 / 3.0)) * divv;
          f[1 + i][k] -= tau;
          work += vel[i] * tau;
        }
        f[NE][k] -= work + kcond * ge[k];
      }
    }
  }
}

template <int D, class V, class R>
__device__ inline V wave_speed(R gam, const V* u, const R* n) {
  using T = VT<V>;
  V rho = u[0], E = u[D + 1];
  V rinv = T::mk(R(1)) / rho;
  V vn = T::mk(R(0)), ke = T::mk(R(0));
#pragma unroll
  for (int k = 0; k < D; ++k) { vn += (u[1 + k] * rinv) * n[k]; ke += u[1 + k] * u[1 + k] * rinv; }
  V pr = (gam - R(1)) * (E - R(0.5) * ke);
  return vabs(vn) + vsqrt(gam * pr * rinv);
}

#ifdef LDG_USER_PHYSICS
template <class U, class = void>
struct UserBou { static constexpr bool value = false; };
template <class U>
struct UserBou<U, typename VoidOf<decltype(U::BOU)>::type> { static constexpr bool value = U::BOU; };
// dependent on U, so that sources without a boundary function never instantiate it
template <class U, int D, class V, class R>
__device__ inline void user_bou(const double* mu, int naux, int tag, const V* uL, const V (*qL)[D], const R* aL,
                                const R* n, V* ub) {
  U::template bou<D, V, R>(mu, naux, tag, uL, qL, aL, n, ub);
}
template <class U, class = void>
struct UserSrc { static constexpr bool value = false; };
template <class U>
struct UserSrc<U, typename VoidOf<decltype(U::SOURCE)>::type> { static constexpr bool value = U::SOURCE; };
template <class U, int D, class V, class R>
__device__ inline void user_source(const double* mu, int naux, const V* u, const V (*q)[D], const R* a, V* s) {
  U::template source<D, V, R>(mu, naux, u, q, a, s);
}
#endif

// state-dependent source s(u, q) of Eq. 1b at a point: a model compiled at run
// time may define one (LdgUser::SOURCE and source<D>); it enters the residual
// as -(s, phi) beside the data source.  false: the model has none.
template <int KIND, int D>
__host__ __device__ constexpr bool has_point_source() {
#ifdef LDG_USER_PHYSICS
  if constexpr (KIND == K_USER) return UserSrc<::LdgUser>::value;
#endif
  return false;
}
template <int KIND, int D, class V, class R>
__device__ inline void point_source(const double* mu, int naux, const V* u, const V (*q)[D], const R* a, V* s) {
#ifdef LDG_USER_PHYSICS
  if constexpr (KIND == K_USER) {
    if constexpr (UserSrc<::LdgUser>::value) user_source<::LdgUser, D, V, R>(mu, naux, u, q, a, s);
  }
#endif
}

// outside state on a Dirichlet-kind boundary face: ub arrives holding the data g.
// A model compiled at run time may define a boundary function (LdgUser::BOU and
// bou<D>), which maps (tag, inside trace, n, g) to the outside state, e.g. a slip
// wall that reverses the normal momentum; for every other model ub stays g.  The
// outside gradient of the numerical flux stays q+ = q-, and the gradient
// equation's boundary trace stays uhat = g (the Dirichlet data).
template <int KIND, int D, class V, class R>
__device__ inline void boundary_state(const double* mu, int naux, int tag, const V* uL, const V (*qL)[D],
                                      const R* aL, const R* n, V* ub) {
#ifdef LDG_USER_PHYSICS
  if constexpr (KIND == K_USER) {
    if constexpr (UserBou<::LdgUser>::value) user_bou<::LdgUser, D, V, R>(mu, naux, tag, uL, qL, aL, n, ub);
  }
#endif
}

// The built-in numerical flux in three pieces, so that a face can finish one
// side's flux before it reads the other side (one dual flux array live at a
// time): Fh (+)= 1/2 f(u, q).n per side, then Fh += sigma (uL - uR).
template <int KIND, int D, class V, class R>
__device__ inline void half_normal_flux(const double* mu, int naux, const V* u, const V (*q)[D], const R* a,
                                        const R* n, V* Fh, bool add) {
  constexpr int NCU = Phys<KIND, D>::NCU;
  V f[NCU][D];
  phys_flux<KIND, D, V, R>(mu, naux, u, q, a, f);
#pragma unroll
  for (int c = 0; c < NCU; ++c) {
    V s = f[c][0] * n[0];
#pragma unroll
    for (int k = 1; k < D; ++k) s += f[c][k] * n[k];
    if (add) Fh[c] += R(0.5) * s;
    else Fh[c] = R(0.5) * s;
  }
}

template <int KIND, int D, class V, class R>
__device__ inline void penalty_flux(const double* mu, const V* uL, const R* aL, const V* uR, const R* aR,
                                    int naux, const R* n, V* Fh) {
  constexpr int NCU = Phys<KIND, D>::NCU;
  if constexpr (KIND == K_POISSON) {
    R kL = naux >= 1 ? aL[0] : R(1), kR = naux >= 1 ? aR[0] : R(1);
    R sig = R(mu[1]) * R(mu[0]) * R(0.5) * (kL + kR);
    Fh[0] += sig * (uL[0] - uR[0]);
  } else if constexpr (KIND == K_CONVDIFF) {
    R sig = R(mu[1]) * R(mu[0]) * R(0.5) * (aL[0] + aR[0]);
    R bnL = R(0), bnR = R(0);
#pragma unroll
    for (int k = 0; k < D; ++k) { bnL += aL[1 + k] * n[k]; bnR += aR[1 + k] * n[k]; }
    sig += R(0.5) * vmax(vabs(bnL), vabs(bnR));
    Fh[0] += sig * (uL[0] - uR[0]);
  } else {
    const R gam = R(mu[0]);
    V lam = vmax(wave_speed<D, V, R>(gam, uL, n), wave_speed<D, V, R>(gam, uR, n));
    V sig = R(0.5) * lam;
    if constexpr (KIND == K_NS) sig = sig + R(mu[3] / mu[1]);
#pragma unroll
    for (int c = 0; c < NCU; ++c) Fh[c] += sig * (uL[c] - uR[c]);
  }
}

// interior numerical flux (also used at Dirichlet faces with u+ = g, q+ = q-, a+ = a-)
template <int KIND, int D, class V, class R>
__device__ inline void num_flux(const double* mu, int naux, const V* uL, const V (*qL)[D], const R* aL,
                                const V* uR, const V (*qR)[D], const R* aR, const R* n, V* Fh) {
#ifdef LDG_USER_PHYSICS
  if constexpr (KIND == K_USER) {
    ::LdgUser::template numflux<D, V, R>(mu, naux, uL, qL, aL, uR, qR, aR, n, Fh);
  } else
#endif
  {
    half_normal_flux<KIND, D, V, R>(mu, naux, uL, qL, aL, n, Fh, false);
    half_normal_flux<KIND, D, V, R>(mu, naux, uR, qR, aR, n, Fh, true);
    penalty_flux<KIND, D, V, R>(mu, uL, aL, uR, aR, naux, n, Fh);
  }
}

}  // namespace ldg
