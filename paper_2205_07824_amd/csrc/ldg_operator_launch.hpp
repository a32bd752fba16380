// Host launchers of the operator kernels and the per-kind entry points.
#pragma once

#include "ldg_internal.hpp"
#include "ldg_operator_kernels.hpp"

namespace ldg {

// ============================================================================
// host dispatch
// ============================================================================
// precision modes of the operator entry points: PM_FP64, PM_FP32 (FP32 arithmetic
// and intermediates, FP64 vectors), PM_FP32_STATE (FP32 arithmetic, FP32 input vectors)
template <int KIND, int D, int P1, class R, class S = double>
static ldg_status launch_grad(const Model& md, const void* uv, void* q, bool with_data, hipStream_t s) {
  const S* u = (const S*)uv;
  // linear models: homogeneous kernel + boundary-data offset; nonlinear: data in the kernel
  const bool in_kernel_data = with_data && !Phys<KIND, D>::LINEAR;
  const double* qoff = (with_data && Phys<KIND, D>::LINEAR) ? md.d_qg : nullptr;
  constexpr int NN = GradCfg<KIND, D, P1, R>::NN, EPB = GradCfg<KIND, D, P1, R>::EPB;
  const Mesh& m = *md.mesh;
  if (q == md.d_dq) {
    md.trt_of = nullptr;
    md.trt_sub = nullptr;
  }
  const int nblk = (int)((m.op_E(0) + EPB - 1) / EPB);
  if (nblk == 0) return LDG_OK;
  const MeshDev mdv = m.dev_op(0);
  typename TabOf<R>::T tab;
  if constexpr (std::is_same<R, double>::value) tab = m.tab; else tab = m.tabf;
  const float* nodu = nullptr;
  constexpr int NFPc = GradCfg<KIND, D, P1, R>::NFP, NFc = GradCfg<KIND, D, P1, R>::NF;
  // FP64 Navier-Stokes tangent of q: with trace storage allocated, also the
  // direction's face traces, which the tangent kernel then reads (tied to this
  // direction and element subset until the next tangent of q).  (The same for
  // the FP32 tangent measured slower: its extra trace writes cost more than the
  // line reads they replace.)
  if constexpr (KIND == K_NS && std::is_same<R, double>::value && std::is_same<S, double>::value &&
                NFc * NFPc >= NN) {
    if (!with_data && md.d_trt && q == md.d_dq && m.batch == 1) {
      ModelDev mod = md.dev();
      mod.trt = md.d_trt;
      if (m.affine)
        hipLaunchKernelGGL((k_grad<KIND, D, P1, R, false, false, true, S, true>), dim3(nblk, m.batch), dim3(EPB * NN), 0, s,
                           mdv, tab, mod, u, (R*)q, qoff, nodu);
      else
        hipLaunchKernelGGL((k_grad<KIND, D, P1, R, false, false, false, S, true>), dim3(nblk, m.batch), dim3(EPB * NN), 0, s,
                           mdv, tab, mod, u, (R*)q, qoff, nodu);
      LDG_TRY(hipGetLastError());
      md.trt_of = uv;
      md.trt_sub = m.sub_list[0];
      return LDG_OK;
    }
  }
  if (in_kernel_data) {
    if (m.affine)
      hipLaunchKernelGGL((k_grad<KIND, D, P1, R, true, false, true, S>), dim3(nblk, m.batch), dim3(EPB * NN), 0, s, mdv, tab,
                         md.dev(), u, (R*)q, qoff, nodu);
    else
      hipLaunchKernelGGL((k_grad<KIND, D, P1, R, true, false, false, S>), dim3(nblk, m.batch), dim3(EPB * NN), 0, s, mdv, tab,
                         md.dev(), u, (R*)q, qoff, nodu);
  } else {
    if (m.affine)
      hipLaunchKernelGGL((k_grad<KIND, D, P1, R, false, false, true, S>), dim3(nblk, m.batch), dim3(EPB * NN), 0, s, mdv, tab,
                         md.dev(), u, (R*)q, qoff, nodu);
    else
      hipLaunchKernelGGL((k_grad<KIND, D, P1, R, false, false, false, S>), dim3(nblk, m.batch), dim3(EPB * NN), 0, s, mdv, tab,
                         md.dev(), u, (R*)q, qoff, nodu);
  }
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

template <int KIND, int D, int P1, class R, int MODE, class S = double>
static ldg_status launch_resid(const Model& md, const TimeDev& t, const void* uv, const void* q, const void* vv,
                               const void* dq, const double* dterm, double* out, hipStream_t s) {
  const S* u = (const S*)uv;
  const S* v = (const S*)vv;
  constexpr int NN = ResidCfg<KIND, D, P1, R, MODE>::NN, EPB = ResidCfg<KIND, D, P1, R, MODE>::EPB;
  const Mesh& m = *md.mesh;
  const int nblk = (int)((m.op_E(1) + EPB - 1) / EPB);
  if (nblk == 0) return LDG_OK;
  const MeshDev mdv = m.dev_op(1);
  typename TabOf<R>::T tab;
  if constexpr (std::is_same<R, double>::value) tab = m.tab; else tab = m.tabf;
  float* noF = nullptr;
  ModelDev mod = md.dev();
  // the tangent reads the face traces of the linearization point when they are
  // formed for u (FP64: for this u; FP32: together with the FP32 q cache it
  // reads), and (FP64) those of the direction when the last tangent of q wrote
  // them for this direction and element subset
  if constexpr (MODE == 2 && KIND == K_NS) {
    bool trc = false, dir = false;
    if constexpr (std::is_same<R, double>::value && std::is_same<S, double>::value) {
      trc = md.d_tr && md.tr_of && md.tr_of == (const double*)uv && md.q_of[0] == (const double*)uv && q == md.d_q;
      dir = trc && md.d_trt && md.trt_of == vv && dq == md.d_dq && md.trt_sub == m.sub_list[0] && m.batch == 1;
      mod.tr = md.d_tr;
      mod.trt = md.d_trt;
    } else if constexpr (std::is_same<R, float>::value) {
      trc = md.d_tr32 && md.tr32_valid && q == md.d_q32;
      mod.tr32 = md.d_tr32;
    }
    (void)dir;
    if constexpr (std::is_same<R, double>::value && std::is_same<S, double>::value) {
      if (dir) {
        if (m.affine)
          hipLaunchKernelGGL((k_resid<KIND, D, P1, R, MODE, false, true, S, true, true>), dim3(nblk, m.batch),
                             dim3(EPB * NN), 0, s, mdv, tab, mod, t, u, (const R*)q, v, (const R*)dq, dterm, out, noF);
        else
          hipLaunchKernelGGL((k_resid<KIND, D, P1, R, MODE, false, false, S, true, true>), dim3(nblk, m.batch),
                             dim3(EPB * NN), 0, s, mdv, tab, mod, t, u, (const R*)q, v, (const R*)dq, dterm, out, noF);
        LDG_TRY(hipGetLastError());
        return LDG_OK;
      }
    }
    if (trc && m.affine && m.probe_nbr) {
      hipLaunchKernelGGL((k_resid<KIND, D, P1, R, MODE, false, true, S, true, false, true>), dim3(nblk, m.batch),
                         dim3(EPB * NN), 0, s, mdv, tab, mod, t, u, (const R*)q, v, (const R*)dq, dterm, out, noF);
      LDG_TRY(hipGetLastError());
      return LDG_OK;
    }
    if (m.probe_nbr) {   // the neighbours' tangent of q was not formed: only the closed form has it
      set_error("block probing with closed-form neighbour traces needs the linearization point's traces");
      return LDG_EINVAL;
    }
    if (trc) {
      if (m.affine)
        hipLaunchKernelGGL((k_resid<KIND, D, P1, R, MODE, false, true, S, true>), dim3(nblk, m.batch), dim3(EPB * NN),
                           0, s, mdv, tab, mod, t, u, (const R*)q, v, (const R*)dq, dterm, out, noF);
      else
        hipLaunchKernelGGL((k_resid<KIND, D, P1, R, MODE, false, false, S, true>), dim3(nblk, m.batch), dim3(EPB * NN),
                           0, s, mdv, tab, mod, t, u, (const R*)q, v, (const R*)dq, dterm, out, noF);
      LDG_TRY(hipGetLastError());
      return LDG_OK;
    }
  }
  if (m.affine)
    hipLaunchKernelGGL((k_resid<KIND, D, P1, R, MODE, false, true, S>), dim3(nblk, m.batch), dim3(EPB * NN), 0, s, mdv, tab,
                       mod, t, u, (const R*)q, v, (const R*)dq, dterm, out, noF);
  else
    hipLaunchKernelGGL((k_resid<KIND, D, P1, R, MODE, false, false, S>), dim3(nblk, m.batch), dim3(EPB * NN), 0, s, mdv, tab,
                       mod, t, u, (const R*)q, v, (const R*)dq, dterm, out, noF);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

template <int KIND, int D, int P1>
static ldg_status launch_grad_ext(const Model& md, const double* u, const float* du, float* q, hipStream_t s) {
  constexpr int NN = GradCfg<KIND, D, P1, float>::NN, EPB = GradCfg<KIND, D, P1, float>::EPB;
  const Mesh& m = *md.mesh;
  const int nblk = (int)((m.E + EPB - 1) / EPB);
  hipLaunchKernelGGL((k_grad<KIND, D, P1, float, false, true>), dim3(nblk), dim3(EPB * NN), 0, s, m.dev(), m.tabf,
                     md.dev(), u, q, (const double*)nullptr, du);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

template <int KIND, int D, int P1>
static ldg_status launch_resid_ext(const Model& md, const TimeDev& t, const double* u, const float* q, float* F,
                                   double* out, hipStream_t s) {
  constexpr int NN = ResidCfg<KIND, D, P1, float, 0>::NN, EPB = ResidCfg<KIND, D, P1, float, 0>::EPB;
  const Mesh& m = *md.mesh;
  const int nblk = (int)((m.E + EPB - 1) / EPB);
  hipLaunchKernelGGL((k_resid<KIND, D, P1, float, 0, true>), dim3(nblk), dim3(EPB * NN), 0, s, m.dev(), m.tabf,
                     md.dev(), t, u, q, (const double*)nullptr, (const float*)nullptr, (const double*)nullptr, out, F);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

// dispatch over (nd, p+1) for one model kind
template <int KI, template <int, int, int> class F, class... Args>
static ldg_status dispatch_kind(int nd, int p1, Args&&... args) {
#define LDG_CASE(DD, PP) \
  if (nd == DD && p1 == PP) return F<KI, DD, PP>::run(args...);
  LDG_CASE(2, 2) LDG_CASE(2, 3) LDG_CASE(2, 4) LDG_CASE(2, 5) LDG_CASE(3, 2) LDG_CASE(3, 3) LDG_CASE(3, 4)
#undef LDG_CASE
  set_error("no compiled kernel for this (model, nd, p)");
  return LDG_EUNSUPPORTED;
}

template <int KI, int DD, int PP>
struct GradOp {
  static ldg_status run(const Model& md, const void* u, void* q, int pm, bool with_data, hipStream_t s) {
    if constexpr (KI == K_EULER) {
      return LDG_OK;
    } else {
      if (pm == PM_FP32_STATE) return launch_grad<KI, DD, PP, float, float>(md, u, q, with_data, s);
      if (pm == PM_FP32) return launch_grad<KI, DD, PP, float>(md, u, q, with_data, s);
      return launch_grad<KI, DD, PP, double>(md, u, q, with_data, s);
    }
  }
};

template <int KI, int DD, int PP>
struct ResidOp {
  static ldg_status run(const Model& md, const TimeDev& t, const void* u, const void* q, double* out, int pm,
                        bool with_data, hipStream_t s) {
    if constexpr (KI <= K_CONVDIFF) {
      const double* dt = with_data ? md.d_dterm : nullptr;
      if (pm == PM_FP32_STATE) {
        if (with_data) { set_error("the FP32-state operator is the linear part only"); return LDG_EINVAL; }
        return launch_resid<KI, DD, PP, float, 0, float>(md, t, u, q, nullptr, nullptr, nullptr, out, s);
      }
      if (pm == PM_FP32) return launch_resid<KI, DD, PP, float, 0>(md, t, u, q, nullptr, nullptr, dt, out, s);
      return launch_resid<KI, DD, PP, double, 0>(md, t, u, q, nullptr, nullptr, dt, out, s);
    } else {
      if (pm == PM_FP32_STATE) { set_error("the residual takes an FP64 state"); return LDG_EINVAL; }
      if (pm == PM_FP32) return launch_resid<KI, DD, PP, float, 1>(md, t, u, q, nullptr, nullptr, nullptr, out, s);
      return launch_resid<KI, DD, PP, double, 1>(md, t, u, q, nullptr, nullptr, nullptr, out, s);
    }
  }
};

template <int KI, int DD, int PP>
struct TangentOp {
  static ldg_status run(const Model& md, const TimeDev& t, const void* u, const void* q, const void* v,
                        const void* dq, double* out, int pm, hipStream_t s) {
    if constexpr (KI <= K_CONVDIFF) {
      set_error("tangent kernel requested for a linear model");
      return LDG_EINVAL;
    } else {
      if (pm == PM_FP32_STATE) return launch_resid<KI, DD, PP, float, 2, float>(md, t, u, q, v, dq, nullptr, out, s);
      if (pm == PM_FP32) return launch_resid<KI, DD, PP, float, 2>(md, t, u, q, v, dq, nullptr, out, s);
      return launch_resid<KI, DD, PP, double, 2>(md, t, u, q, v, dq, nullptr, out, s);
    }
  }
};

template <int KI, int DD, int PP>
struct GradExtOp {
  static ldg_status run(const Model& md, const double* u, const float* du, float* q, hipStream_t s) {
    if constexpr (KI <= K_CONVDIFF) return launch_grad_ext<KI, DD, PP>(md, u, du, q, s);
    else { set_error("external contractions are for the linear models"); return LDG_EUNSUPPORTED; }
  }
};
template <int KI, int DD, int PP>
struct ResidExtOp {
  static ldg_status run(const Model& md, const TimeDev& t, const double* u, const float* q, float* F, double* out,
                        hipStream_t s) {
    if constexpr (KI <= K_CONVDIFF) return launch_resid_ext<KI, DD, PP>(md, t, u, q, F, out, s);
    else { set_error("external contractions are for the linear models"); return LDG_EUNSUPPORTED; }
  }
};

// per-kind entry points, defined in ldg_op_<kind>.hip
template <int KI> struct KindOps {
  static ldg_status grad(const Model& md, const void* u, void* q, int pm, bool with_data, hipStream_t s);
  static ldg_status resid(const Model& md, const TimeDev& t, const void* u, const void* q, double* out, int pm,
                          bool with_data, hipStream_t s);
  static ldg_status tangent(const Model& md, const TimeDev& t, const void* u, const void* q, const void* v,
                            const void* dq, double* out, int pm, hipStream_t s);
  static ldg_status grad_ext(const Model& md, const double* u, const float* du, float* q, hipStream_t s);
  static ldg_status resid_ext(const Model& md, const TimeDev& t, const double* u, const float* q, float* F,
                              double* out, hipStream_t s);
};

#define LDG_DEFINE_KIND_OPS(KI)                                                                                  \
  template <> ldg_status KindOps<KI>::grad(const Model& md, const void* u, void* q, int pm, bool with_data,      \
                                           hipStream_t s) {                                                      \
    return dispatch_kind<KI, GradOp>(md.mesh->nd, md.mesh->p1, md, u, q, pm, with_data, s);                      \
  }                                                                                                              \
  template <> ldg_status KindOps<KI>::resid(const Model& md, const TimeDev& t, const void* u, const void* q,     \
                                            double* out, int pm, bool with_data, hipStream_t s) {                \
    return dispatch_kind<KI, ResidOp>(md.mesh->nd, md.mesh->p1, md, t, u, q, out, pm, with_data, s);             \
  }                                                                                                              \
  template <> ldg_status KindOps<KI>::tangent(const Model& md, const TimeDev& t, const void* u, const void* q,   \
                                              const void* v, const void* dq, double* out, int pm,                \
                                              hipStream_t s) {                                                   \
    return dispatch_kind<KI, TangentOp>(md.mesh->nd, md.mesh->p1, md, t, u, q, v, dq, out, pm, s);               \
  }                                                                                                              \
  template <> ldg_status KindOps<KI>::grad_ext(const Model& md, const double* u, const float* du, float* q,      \
                                               hipStream_t s) {                                                  \
    return dispatch_kind<KI, GradExtOp>(md.mesh->nd, md.mesh->p1, md, u, du, q, s);                              \
  }                                                                                                              \
  template <> ldg_status KindOps<KI>::resid_ext(const Model& md, const TimeDev& t, const double* u, const float* q, \
                                                float* F, double* out, hipStream_t s) {                          \
    return dispatch_kind<KI, ResidExtOp>(md.mesh->nd, md.mesh->p1, md, t, u, q, F, out, s);                      \
  }

}  // namespace ldg
