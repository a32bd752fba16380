// Internal definitions of the host code (the device-side ones are in ldg_device.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ldg.h"
#include "ldg_device.hpp"

namespace ldg {

static_assert((int)BC_DIRICHLET == (int)LDG_BC_DIRICHLET && (int)BC_NEUMANN == (int)LDG_BC_NEUMANN &&
                  (int)BC_EXTRAP == (int)LDG_BC_EXTRAP,
              "device boundary kinds are the ABI's");

// --------------------------------------------------------------------------
// Host-side objects
// --------------------------------------------------------------------------
struct Mesh {
  int nd, p, nq1, p1, nn, nqv, nqf, nfp, nv, nf;
  int64_t E, nbf;
  bool affine;
  BasisTab tab;
  BasisTabF tabf;
  std::vector<double> h_coef;         // [E][nv][nd]
  std::vector<int32_t> h_nbr;         // [E][nf]
  std::vector<int64_t> h_bface;       // [nbf][2]
  std::vector<int32_t> h_btag;        // [nbf]
  std::vector<int32_t> h_color;       // [E]
  int ncolors;
  std::vector<std::vector<int32_t>> color_elems;
  // quadrature rule with nq1 points (data terms)
  std::vector<double> xq1, wq1;
  double* d_coef = nullptr;
  int32_t* d_nbr = nullptr;
  int32_t* d_btag = nullptr;
  int32_t* d_color_list = nullptr;    // elements sorted by colour
  std::vector<int32_t> h_order;       // [E] Morton order of the element centroids
  int32_t* d_order = nullptr;
  std::vector<int64_t> color_off;     // [ncolors+1] offsets into d_color_list
  int32_t* d_color_nbhd = nullptr;    // per colour: its elements and their face neighbours, sorted
  std::vector<int64_t> nbhd_off;      // [ncolors+1] offsets into d_color_nbhd
  // Element subsets of the operator launches ([0] gradient kernels, [1]
  // residual / tangent kernels; nullptr = every element).  Block probing sets
  // them: a JVP seeded on one colour needs its rows only on that colour, and
  // the tangent of q only on the colour and its face neighbours.
  const int32_t* sub_list[2] = {nullptr, nullptr};
  int64_t sub_count[2] = {0, 0};
  MeshDev dev() const { return MeshDev{(int)E, (int)nbf, d_coef, d_nbr, d_btag, d_order}; }
  // products batched over blockIdx.y (set with the subsets by the block probing)
  int batch = 1;
  int64_t bsn = 0, bsq = 0;
  // every element's face neighbours are distinct elements other than itself
  // (no element touches another across two faces, as on 1- or 2-element-wide
  // periodic meshes); the probing's closed-form neighbour traces need it
  bool nbr_distinct = false;
  // block probing on such an affine mesh, with the linearization point's traces
  // formed: the tangent kernel forms the neighbours' tangent-of-q traces in
  // closed form from its own direction trace, and the gradient pass runs on
  // the seeded colour alone
  bool probe_nbr = false;
  MeshDev dev_op(int which) const {
    MeshDev r = sub_list[which] ? MeshDev{(int)sub_count[which], (int)nbf, d_coef, d_nbr, d_btag, sub_list[which]}
                                : dev();
    if (batch > 1) { r.bsn = bsn; r.bsq = bsq; }
    return r;
  }
  int64_t op_E(int which) const { return sub_list[which] ? sub_count[which] : E; }
};

struct JitOps;   // run-time compiled physics (ldg_jit.hip)
struct MfmaWork; // operators of the MFMA product (ldg_mfma.hip)

struct Model {
  Mesh* mesh;
  int kind, ncu, nmu, naux;
  double mu[MAXMU];
  int nbc;
  int bc_kind[MAXTAG];
  const double* aux;     // caller's device arrays
  const double* src;
  const double* bdata;
  bool linear;
  bool hasq = true;           // the model's flux depends on q (all but Euler)
  JitOps* jit = nullptr;      // kernels of a model compiled at run time
  MfmaWork* mfma = nullptr;   // operators of the MFMA product (linear models)
  double* d_qg = nullptr;     // linear models: q offset from boundary data  [E][ncu][nd][nn]
  double* d_dterm = nullptr;  // linear models: data terms of the residual   [E][ncu][nn]
  double* d_srcn = nullptr;   // nonlinear models: source at nodes          [E][ncu][nn]
  // workspace
  double* d_q = nullptr;      // q(u_lin) cache of the linearization point, FP64
  float* d_q32 = nullptr;     // the same in FP32 (mixed-precision tangents)
  double* d_qres = nullptr;   // q of residual evaluations
  void* d_dq = nullptr;       // tangent of q (FP64 or FP32)
  double* d_tmp = nullptr;    // vector-size scratch (FD JVP, linearization)
  double* d_tmp2 = nullptr;
  double* d_red = nullptr;    // reduction scratch (4096 doubles)
  const double* q_of[2] = {nullptr, nullptr};   // state whose q sits in d_q / d_q32 (ldg_jvp_prepared checks it)
  double* d_tr = nullptr;       // face traces of (u, q(u)) of the FP64 linearization point (Navier-Stokes)
  const double* tr_of = nullptr;  // the state whose traces sit in d_tr
  float* d_tr32 = nullptr;        // the same in FP32, formed with d_q32
  double* d_trt = nullptr;        // FP64 traces of the last product's direction
  // the direction and element subset whose traces were last written
  mutable const void* trt_of = nullptr;
  mutable const int32_t* trt_sub = nullptr;
  bool tr32_valid = false;        // d_tr32 holds the traces of the state whose q sits in d_q32
  double* d_probe = nullptr;      // batched probing vectors (direction, result, tangent of q), per batch entry
  int probe_batch = 0;            // batch entries d_probe holds
  size_t N() const { return (size_t)mesh->E * ncu * mesh->nn; }
  ModelDev dev() const {
    ModelDev d{};
    for (int i = 0; i < MAXMU; ++i) d.mu[i] = mu[i];
    d.naux = naux; d.aux = aux; d.src = d_srcn; d.bdata = bdata;
    for (int i = 0; i < MAXTAG; ++i) d.bc_kind[i] = bc_kind[i];
    d.nbc = nbc;
    return d;
  }
};

// zero a device int (a kernel, so the call is safe inside captured graphs)
ldg_status zero_int(int* p, hipStream_t s);

// status helpers
void set_error(const std::string& msg);
// entry of every ABI call: drop a stale error left by unrelated HIP calls, so
// that the launch checks below report only this call's own failures
#define LDG_ENTER() (void)hipGetLastError()
#define LDG_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      ::ldg::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));         \
      return LDG_EDEVICE;                                                          \
    }                                                                              \
  } while (0)

// precision modes of the operator entry points: FP64; FP32 arithmetic and
// intermediates with FP64 input vectors; FP32 arithmetic with FP32 input vectors
// (u, v; the output stays FP64).  A bool argument converts to the first two.
enum PrecMode { PM_FP64 = 0, PM_FP32 = 1, PM_FP32_STATE = 2 };

// operator entry points (ldg_operator.hip); u and v are double, or float under PM_FP32_STATE
ldg_status op_grad(const Model& md, const void* u, void* q, int pm, bool with_data, hipStream_t s);
ldg_status op_resid(const Model& md, const TimeDev& t, const void* u, const void* q, double* out, int pm,
                    bool with_data, hipStream_t s);
ldg_status op_jvp_nonlinear(const Model& md, const TimeDev& t, const void* u, const void* q, const void* v,
                            const void* dq, double* out, int pm, hipStream_t s);
ldg_status op_data_terms(Model& md, hipStream_t s);
// q(u) of an FP64 linearization point into md.d_q (and, for the models whose
// tangent kernels read them, the face traces of u and q(u) into md.d_tr);
// sets md.q_of[0] (and md.tr_of) to u
ldg_status form_q_cache64(Model& md, const double* u, hipStream_t s);
// q(u) in FP32 into md.d_q32 and, for the Navier-Stokes tangent, its face traces
// into md.d_tr32; u is double (pm = PM_FP32) or float (pm = PM_FP32_STATE);
// md.q_of[1] becomes u for a double u, nullptr for a float one
ldg_status form_q_cache32(Model& md, const void* u, int pm, hipStream_t s);
ldg_status op_mfma_jvp(const Model& md, const TimeDev& t, const double* v, double* out, bool fp16, hipStream_t s);
ldg_status mfma_prepare(Model& md);
void mfma_release(Model& md);

// run-time compiled physics (ldg_jit.hip)
ldg_status jit_build(Model& md, const char* user_source);
void jit_release(Model& md);
ldg_status jit_check(const char* user_source, int nd, int p1, int ncu, bool hasq);
ldg_status jit_grad(const Model& md, const double* u, void* q, bool fp32, bool with_data, hipStream_t s);
ldg_status jit_resid(const Model& md, const TimeDev& t, const double* u, const void* q, const double* v,
                     const void* dq, double* out, bool fp32, bool tangent, hipStream_t s);
int jit_ode_size(const Model& md);
ldg_status jit_ode(const Model& md, const TimeDev& t, double alpha, double beta, const double* u, double* w,
                   hipStream_t s);

// shared host helpers (ldg_api.hip)
TimeDev make_time(const ldg_time* t, bool with_rhs);
ldg_status residual_impl(Model& md, const ldg_time* t, const double* u, double* G, double* q_out, bool fp32,
                         hipStream_t s);
ldg_status jvp_state32(Model& md, const ldg_time* t, const float* u, const float* v, double* Jv, bool prepared,
                       hipStream_t s);
ldg_status jvp_impl(Model& md, const ldg_time* t, const double* u, const double* v, double* Jv, ldg_precision prec,
                    bool prepared, hipStream_t s);

// vector kernels (ldg_krylov.hip)
ldg_status vec_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
ldg_status vec_fill(int64_t n, double a, double* y, hipStream_t s);
// host result of sum(x*x); uses a small device scratch owned by the caller
ldg_status vec_norm2(int64_t n, const double* x, double* partial, double* host_out, hipStream_t s);

}  // namespace ldg

// opaque ABI handles are the internal objects
struct ldg_mesh_s : public ldg::Mesh {};
struct ldg_model_s : public ldg::Model {};
