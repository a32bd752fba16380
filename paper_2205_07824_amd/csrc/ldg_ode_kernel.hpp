// The ODE that the paper couples to the PDE (Eq. 1c): alpha dw/dt + beta w = s_w,
// with w (n_w components) carried at the element nodes beside the PDE state and
// s_w a pointwise function of the state.  Compiled at run time with the model's
// physics (struct LdgUser: NW and ode_source); a physics source without NW has
// no ODE and this kernel does nothing.
//
// One implicit stage of the time wrapper (w_t ~ a0 w - (c1 r1 + c2 r2), the same
// wrapper as the PDE's) is linear in w and local to each node:
//     alpha (a0 w - c1 r1 - c2 r2) + beta w = s_w(u)
//  => w = (alpha (c1 r1 + c2 r2) + s_w(u)) / (alpha a0 + beta).
#pragma once

#include "ldg_device.hpp"

namespace ldg {

template <class U, class = void>
struct UserOde {
  static constexpr int NW = 0;
  __device__ static void source(const double*, int, const double*, const double*, double*) {}
};

template <class U>
struct UserOde<U, typename VoidOf<decltype(U::NW)>::type> {
  static constexpr int NW = U::NW;
  static_assert(NW >= 1 && NW <= 8, "LdgUser::NW must be in [1, 8]");
  __device__ static void source(const double* mu, int naux, const double* u, const double* a, double* sw) {
    U::ode_source(mu, naux, u, a, sw);
  }
};

}  // namespace ldg

// number of ODE components, read by the host after loading the module
extern "C" __device__ int ldg_user_nw = ldg::UserOde<LdgUser>::NW;

// one thread per (element, node); u: [E][NCU][nn], aux: [E][naux][nn], r1, r2, w: [E][NW][nn]
extern "C" __global__ __launch_bounds__(256) void ldg_k_ode_stage(int64_t nodes, int nn, ldg::ModelDev md,
                                                                   double alpha, double beta, double a0, double c1,
                                                                   const double* r1, double c2, const double* r2,
                                                                   const double* u, double* w) {
  using O = ldg::UserOde<LdgUser>;
  constexpr int NCU = LdgUser::NCU;
  constexpr int NA = LdgUser::NAUX > 0 ? LdgUser::NAUX : 1;
  constexpr int NW = O::NW > 0 ? O::NW : 1;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (O::NW == 0 || g >= nodes) return;
  const int64_t K = g / nn;
  const int i = (int)(g - K * nn);
  double uu[NCU], aa[NA], sw[NW];
  for (int c = 0; c < NCU; ++c) uu[c] = u[(K * NCU + c) * nn + i];
  for (int t = 0; t < NA; ++t) aa[t] = t < md.naux ? md.aux[(K * md.naux + t) * nn + i] : 0.0;
  O::source(md.mu, md.naux, uu, aa, sw);
  const double den = alpha * a0 + beta;
  for (int m = 0; m < NW; ++m) {
    const int64_t off = (K * NW + m) * nn + i;
    double rhs = 0.0;
    if (r1) rhs += c1 * r1[off];
    if (r2) rhs += c2 * r2[off];
    w[off] = (alpha * rhs + sw[m]) / den;
  }
}
