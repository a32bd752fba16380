// Model-kind dispatch of the operator kernels, and the set-up kernel that
// integrates the data terms of the linear models.
#include "ldg_operator_launch.hpp"

namespace ldg {

// ============================================================================
// Data terms of the linear models, integrated with the nq1-point rule (set-up
// only, once per model):
//   qg[c][k](i)  = -(1 / (w_i |J(x_i)|)) sum_{Dirichlet faces} <g n_k, phi_i>
//   dterm[c](i)  = <Fhat_data, phi_i> - (s, phi_i)
// with Fhat_data = (1/2 b.n - sigma) g on Dirichlet faces (sigma as in the
// interior flux with both sides equal) and the flux data h on Neumann faces.
// One thread per (element, node); plain loops over the quadrature points.
// ============================================================================
__device__ inline double lag1(const double* x, int P1, int mI, double t) {
  double r = 1.0;
  for (int j = 0; j < P1; ++j)
    if (j != mI) r *= (t - x[j]) / (x[mI] - x[j]);
  return r;
}

template <int D>
__global__ void k_data_terms(MeshDev m, BasisTab tab, ModelDev md, int kind, int P1, int Q1, const double* xq,
                             const double* wq, const double* __restrict__ src, double* __restrict__ qg,
                             double* __restrict__ dterm) {
  const int nn = (D == 2) ? P1 * P1 : P1 * P1 * P1;
  const int nqf = (D == 2) ? Q1 : Q1 * Q1;
  const int nqv = nqf * Q1;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)m.E * nn) return;
  const int64_t K = g / nn;
  const int i = g % nn;
  constexpr int NV = 1 << D;
  const double* c = m.coef + K * NV * D;
  int a[D];
  {
    int t = i;
    for (int k = 0; k < D; ++k) { a[k] = t % P1; t /= P1; }
  }
  // mass at node i
  double xin[D];
  double wi = 1.0;
  for (int k = 0; k < D; ++k) { xin[k] = tab.x[a[k]]; wi *= tab.w[a[k]]; }
  double Jn[D][D], adjn[D][D];
  jacobian_at<D, double>(c, xin, Jn);
  const double detn = adjugate<D, double>(Jn, adjn);
  const double Mii = wi * detn;

  double qacc[D];
  for (int k = 0; k < D; ++k) qacc[k] = 0.0;
  double dacc = 0.0;
  // volume source
  if (src) {
    for (int qp = 0; qp < nqv; ++qp) {
      int iq[D];
      int t = qp;
      double xi[D], w = 1.0, phi = 1.0;
      for (int k = 0; k < D; ++k) { iq[k] = t % Q1; t /= Q1; xi[k] = xq[iq[k]]; w *= wq[iq[k]]; }
      for (int k = 0; k < D; ++k) phi *= lag1(tab.x, P1, a[k], xi[k]);
      double J[D][D], adj[D][D];
      jacobian_at<D, double>(c, xi, J);
      const double det = adjugate<D, double>(J, adj);
      dacc -= w * det * src[K * nqv + qp] * phi;
    }
  }
  // faces
  for (int F = 0; F < 2 * D; ++F) {
    const int nb = m.nbr[K * 2 * D + F];
    if (nb >= 0) continue;
    const int b = -(nb + 1);
    int tag = m.btag[b];
    tag = tag < 0 ? 0 : (tag >= md.nbc ? md.nbc - 1 : tag);
    const int bk = md.bc_kind[tag];
    if (bk == LDG_BC_EXTRAP || !md.bdata) continue;
    const int dir = F >> 1, side = F & 1;
    const double phin = lag1(tab.x, P1, a[dir], side ? 1.0 : -1.0);
    if (phin == 0.0) continue;
    for (int f = 0; f < nqf; ++f) {
      double xi[D], w = 1.0, phi = phin;
      int ff = f;
      for (int k = 0; k < D; ++k) {
        if (k == dir) { xi[k] = side ? 1.0 : -1.0; continue; }
        const int it = ff % Q1;
        ff /= Q1;
        xi[k] = xq[it];
        w *= wq[it];
        phi *= lag1(tab.x, P1, a[k], xi[k]);
      }
      double J[D][D], N[D];
      jacobian_at<D, double>(c, xi, J);
      scaled_normal<D, double>(J, dir, side, N);
      double ds = 0.0;
      for (int k = 0; k < D; ++k) ds += N[k] * N[k];
      ds = sqrt(ds);
      const double gval = md.bdata[(int64_t)b * nqf + f];
      if (bk == LDG_BC_NEUMANN) {
        dacc += w * ds * gval * phi;
        continue;
      }
      // Dirichlet: aux at the face point
      double kap = 1.0, bn = 0.0;
      if (md.naux >= 1) {
        double av[1 + D];
        for (int t = 0; t < md.naux && t < 1 + D; ++t) {
          double s = 0.0;
          for (int j = 0; j < nn; ++j) {
            int aj[D];
            int tt = j;
            double ph = 1.0;
            for (int k = 0; k < D; ++k) { aj[k] = tt % P1; tt /= P1; ph *= lag1(tab.x, P1, aj[k], xi[k]); }
            s += md.aux[(K * md.naux + t) * nn + j] * ph;
          }
          av[t] = s;
        }
        kap = av[0];
        if (kind == K_CONVDIFF)
          for (int k = 0; k < D; ++k) bn += av[1 + k] * N[k] / ds;
      }
      double sig = md.mu[1] * md.mu[0] * kap;
      if (kind == K_CONVDIFF) sig += 0.5 * (bn >= 0 ? bn : -bn);
      dacc += w * ds * (0.5 * bn - sig) * gval * phi;
      for (int k = 0; k < D; ++k) qacc[k] -= w * gval * N[k] * phi;
    }
  }
  for (int k = 0; k < D; ++k) qg[(K * D + k) * nn + i] = qacc[k] / Mii;
  dterm[K * nn + i] = dacc;
}


template <class F0, class F1, class F2, class F3, class... Args>
static ldg_status by_kind(int kind, F0 f0, F1 f1, F2 f2, F3 f3, Args&&... args) {
  switch (kind) {
    case 0: return f0(args...);
    case 1: return f1(args...);
    case 2: return f2(args...);
    case 3: return f3(args...);
  }
  set_error("unknown model kind");
  return LDG_EINVAL;
}

static ldg_status no_state32_for_user(const Model& md, int pm) {
  if (md.kind == LDG_MODEL_USER && pm == PM_FP32_STATE) {
    set_error("FP32-state products are built for the library's own models, not for run-time physics");
    return LDG_EUNSUPPORTED;
  }
  return LDG_OK;
}

ldg_status op_grad(const Model& md, const void* u, void* q, int pm, bool with_data, hipStream_t s) {
  if (ldg_status st = no_state32_for_user(md, pm)) return st;
  if (md.kind == LDG_MODEL_USER) return jit_grad(md, (const double*)u, q, pm == PM_FP32, with_data, s);
  return by_kind(md.kind, KindOps<0>::grad, KindOps<1>::grad, KindOps<2>::grad, KindOps<3>::grad, md, u, q, pm,
                 with_data, s);
}

ldg_status op_resid(const Model& md, const TimeDev& t, const void* u, const void* q, double* out, int pm,
                    bool with_data, hipStream_t s) {
  if (ldg_status st = no_state32_for_user(md, pm)) return st;
  if (md.kind == LDG_MODEL_USER)
    return jit_resid(md, t, (const double*)u, q, nullptr, nullptr, out, pm == PM_FP32, false, s);
  return by_kind(md.kind, KindOps<0>::resid, KindOps<1>::resid, KindOps<2>::resid, KindOps<3>::resid, md, t, u, q,
                 out, pm, with_data, s);
}

ldg_status op_jvp_nonlinear(const Model& md, const TimeDev& t, const void* u, const void* q, const void* v,
                            const void* dq, double* out, int pm, hipStream_t s) {
  if (ldg_status st = no_state32_for_user(md, pm)) return st;
  if (md.kind == LDG_MODEL_USER)
    return jit_resid(md, t, (const double*)u, q, (const double*)v, dq, out, pm == PM_FP32, true, s);
  return by_kind(md.kind, KindOps<0>::tangent, KindOps<1>::tangent, KindOps<2>::tangent, KindOps<3>::tangent, md, t,
                 u, q, v, dq, out, pm, s);
}

ldg_status op_grad_ext(const Model& md, const double* u, const float* du, float* q, hipStream_t s) {
  return by_kind(md.kind, KindOps<0>::grad_ext, KindOps<1>::grad_ext, KindOps<2>::grad_ext, KindOps<3>::grad_ext, md,
                 u, du, q, s);
}

ldg_status op_resid_ext(const Model& md, const TimeDev& t, const double* u, const float* q, float* F, double* out,
                        hipStream_t s) {
  return by_kind(md.kind, KindOps<0>::resid_ext, KindOps<1>::resid_ext, KindOps<2>::resid_ext, KindOps<3>::resid_ext,
                 md, t, u, q, F, out, s);
}

// face traces of (u, q(u)) for the Navier-Stokes tangent (nd + 2 conserved variables):
// FP64 from md.d_q into md.d_tr, or FP32 from md.d_q32 into md.d_tr32 (u double or float)
template <class R, class S>
static ldg_status launch_face_traces(const Model& md, const S* u, const R* q, R* tr, hipStream_t s) {
  const Mesh& m = *md.mesh;
  const int64_t items = m.E * 2 * m.nd * (m.nd == 3 ? m.p1 * m.p1 : m.p1);
  const unsigned nblk = (unsigned)((items + 255) / 256);
  if (nblk == 0) return LDG_OK;
  typename TabOf<R>::T tab;
  if constexpr (std::is_same<R, double>::value) tab = m.tab; else tab = m.tabf;
#define LDG_TR(DD, PP)                                                                                           \
  if (m.nd == DD && m.p1 == PP) {                                                                                \
    hipLaunchKernelGGL((k_face_traces<DD, PP, DD + 2, R, S>), dim3(nblk), dim3(256), 0, s, m.E, tab, u, q, tr); \
    LDG_TRY(hipGetLastError());                                                                                  \
    return LDG_OK;                                                                                               \
  }
  LDG_TR(2, 2) LDG_TR(2, 3) LDG_TR(2, 4) LDG_TR(2, 5) LDG_TR(3, 2) LDG_TR(3, 3) LDG_TR(3, 4)
#undef LDG_TR
  set_error("no face-trace kernel for this (nd, p)");
  return LDG_EUNSUPPORTED;
}

static int64_t trace_count(const Model& md) {
  const Mesh& m = *md.mesh;
  return m.E * 2 * m.nd * (m.nd == 3 ? m.p1 * m.p1 : m.p1) * (int64_t)md.ncu * (1 + m.nd);
}

// the FP64 traces of the linearization point and of the direction, both or neither
static bool alloc_trace_pair(const Model& md, double** tr, double** trt) {
  const size_t bytes = sizeof(double) * trace_count(md);
  if (hipMalloc((void**)tr, bytes) == hipSuccess) {
    if (hipMalloc((void**)trt, bytes) == hipSuccess) return true;
    (void)hipFree(*tr);
  }
  (void)hipGetLastError();
  *tr = nullptr;
  *trt = nullptr;
  return false;
}

ldg_status form_q_cache64(Model& md, const double* u, hipStream_t s) {
  md.q_of[0] = nullptr;
  md.tr_of = nullptr;
  ldg_status st = op_grad(md, u, md.d_q, PM_FP64, true, s);
  if (st != LDG_OK) return st;
  md.q_of[0] = u;
  if (md.kind != K_NS) return LDG_OK;   // the models whose FP64 tangent kernel reads the traces
  if (!md.d_tr && !alloc_trace_pair(md, &md.d_tr, &md.d_trt))
    return LDG_OK;   // without the traces the tangent kernel reads the neighbours' lines
  st = launch_face_traces<double, double>(md, u, md.d_q, md.d_tr, s);
  if (st != LDG_OK) return st;
  md.tr_of = u;
  return LDG_OK;
}

ldg_status form_q_cache32(Model& md, const void* u, int pm, hipStream_t s) {
  md.q_of[1] = nullptr;
  md.tr32_valid = false;
  ldg_status st = op_grad(md, u, md.d_q32, pm, true, s);
  if (st != LDG_OK) return st;
  if (pm == PM_FP32) md.q_of[1] = (const double*)u;
  if (md.kind != K_NS) return LDG_OK;
  if (!md.d_tr32 && hipMalloc((void**)&md.d_tr32, sizeof(float) * trace_count(md)) != hipSuccess) {
    (void)hipGetLastError();
    md.d_tr32 = nullptr;
    return LDG_OK;
  }
  st = pm == PM_FP32_STATE ? launch_face_traces<float, float>(md, (const float*)u, md.d_q32, md.d_tr32, s)
                           : launch_face_traces<float, double>(md, (const double*)u, md.d_q32, md.d_tr32, s);
  if (st != LDG_OK) return st;
  md.tr32_valid = true;
  return LDG_OK;
}

// data terms of the linear models (qg, dterm), then fold qg into the stored
// offset used by the gradient kernel
ldg_status op_data_terms(Model& md, hipStream_t s) {
  Mesh& m = *md.mesh;
  double *d_xq = nullptr, *d_wq = nullptr;
  LDG_TRY(hipMalloc((void**)&d_xq, sizeof(double) * m.nq1));
  LDG_TRY(hipMalloc((void**)&d_wq, sizeof(double) * m.nq1));
  LDG_TRY(hipMemcpyAsync(d_xq, m.xq1.data(), sizeof(double) * m.nq1, hipMemcpyHostToDevice, s));
  LDG_TRY(hipMemcpyAsync(d_wq, m.wq1.data(), sizeof(double) * m.nq1, hipMemcpyHostToDevice, s));
  const int64_t tot = m.E * m.nn;
  const int nb = (int)((tot + 127) / 128);
  ModelDev dv = md.dev();
  if (m.nd == 2)
    hipLaunchKernelGGL(k_data_terms<2>, dim3(nb), dim3(128), 0, s, m.dev(), m.tab, dv, md.kind, m.p1, m.nq1, d_xq,
                       d_wq, md.src, md.d_qg, md.d_dterm);
  else
    hipLaunchKernelGGL(k_data_terms<3>, dim3(nb), dim3(128), 0, s, m.dev(), m.tab, dv, md.kind, m.p1, m.nq1, d_xq,
                       d_wq, md.src, md.d_qg, md.d_dterm);
  LDG_TRY(hipGetLastError());
  LDG_TRY(hipStreamSynchronize(s));
  LDG_TRY(hipFree(d_xq));
  LDG_TRY(hipFree(d_wq));
  return LDG_OK;
}

}  // namespace ldg
