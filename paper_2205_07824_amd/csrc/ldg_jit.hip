// Models whose pointwise physics is compiled at run time.  The paper generates
// the flux, source and boundary code of each PDE from its symbolic description
// (Section 3); here the caller hands over a C++ source of the pointwise physics
// (struct LdgUser: flux and numerical flux, written once for values and dual
// numbers), and hipRTC compiles it together with the library's own operator
// kernels for the mesh's element type and order.  The tangent kernels
// differentiate the user's arithmetic exactly, as for the built-in models.
#include <hip/hiprtc.h>

#include <cstring>
#include <string>
#include <vector>

#include "ldg_internal.hpp"
#include "ldg_operator_kernels.hpp"
#include "ldg_jit_sources.inc"   // generated at build time: the device headers as string literals

namespace ldg {

struct JitOps {
  hipModule_t mod = nullptr;
  hipFunction_t grad[2][2] = {};   // [FP32][with boundary data]
  hipFunction_t resid[2][2] = {};  // [FP32][tangent]
  int epb_grad[2] = {0, 0};
  int epb_resid[2][2] = {{0, 0}, {0, 0}};
  hipFunction_t ode = nullptr;     // one implicit stage of the coupled ODE (Eq. 1c)
  int nw = 0;                      // its number of components (0: the source defines no ODE)
};

namespace {

std::string program_text(const char* user, int ncu, bool hasq) {
  std::string p;
  p += "#define LDG_USER_PHYSICS 1\n#include \"ldg_device.hpp\"\nusing namespace ldg;\n";
  p += "#line 1 \"physics_source\"\n";
  p += user;
  p += "\n#include \"ldg_operator_kernels.hpp\"\n#include \"ldg_ode_kernel.hpp\"\n";
  p += "static_assert(LdgUser::NCU == " + std::to_string(ncu) + ", \"LdgUser::NCU differs from the model's ncu\");\n";
  p += std::string("static_assert(LdgUser::HASQ == ") + (hasq ? "true" : "false") +
       ", \"LdgUser::HASQ differs from has_q\");\n";
  // the kernels stage max(NAUX, 1) aux values per point: the host reads the bound back
  p += "extern \"C\" __device__ int ldg_user_naux = LdgUser::NAUX;\n";
  return p;
}

// kernel instances, in the order [grad: FP64 no data, FP64 data, FP32 no data, FP32 data]
// [resid: FP64 residual, FP64 tangent, FP32 residual, FP32 tangent]
std::vector<std::string> kernel_names(int nd, int p1, bool aff) {
  std::vector<std::string> v;
  const std::string tail = std::string(", false, ") + (aff ? "true" : "false") + ">";
  const std::string dp = std::to_string(nd) + ", " + std::to_string(p1);
  for (const char* r : {"double", "float"})
    for (const char* data : {"false", "true"})
      v.push_back(std::string("ldg::k_grad<4, ") + dp + ", " + r + ", " + data + tail);
  for (const char* r : {"double", "float"})
    for (const char* mode : {"1", "2"})
      v.push_back(std::string("ldg::k_resid<4, ") + dp + ", " + r + ", " + mode + tail);
  return v;
}

ldg_status compile(const char* user, int nd, int p1, bool aff, int ncu, bool hasq, std::vector<char>* code,
                   std::vector<std::string>* lowered) {
  const std::string text = program_text(user, ncu, hasq);
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, text.c_str(), "ldg_user_physics.hip", kJitHeaderCount, kJitHeaderSources,
                          kJitHeaderNames) != HIPRTC_SUCCESS) {
    set_error("hipRTC could not create the program");
    return LDG_EDEVICE;
  }
  const std::vector<std::string> names = kernel_names(nd, p1, aff);
  for (const auto& n : names) hiprtcAddNameExpression(prog, n.c_str());
  // the same code generation flags as the library's own kernels (no packed FP32 instructions)
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    std::string log;
    if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
      log.resize(n);
      hiprtcGetProgramLog(prog, &log[0]);
    }
    hiprtcDestroyProgram(&prog);
    set_error("physics source does not compile:\n" + log);
    return LDG_EINVAL;
  }
  size_t sz = 0;
  ldg_status st = LDG_OK;
  if (code) {
    if (hiprtcGetCodeSize(prog, &sz) != HIPRTC_SUCCESS) st = LDG_EDEVICE;
    if (st == LDG_OK) {
      code->resize(sz);
      if (hiprtcGetCode(prog, code->data()) != HIPRTC_SUCCESS) st = LDG_EDEVICE;
    }
  }
  if (lowered)
    for (const auto& n : names) {
      const char* low = nullptr;
      if (hiprtcGetLoweredName(prog, n.c_str(), &low) != HIPRTC_SUCCESS || !low) { st = LDG_EDEVICE; break; }
      lowered->push_back(low);
    }
  hiprtcDestroyProgram(&prog);
  if (st != LDG_OK) set_error("hipRTC did not return the compiled kernels");
  return st;
}

}  // namespace

ldg_status jit_build(Model& md, const char* user) {
  const Mesh& m = *md.mesh;
  std::vector<char> code;
  std::vector<std::string> low;
  ldg_status st = compile(user, m.nd, m.p1, m.affine, md.ncu, md.hasq, &code, &low);
  if (st != LDG_OK) return st;
  auto* J = new JitOps();
  if (hipModuleLoadData(&J->mod, code.data()) != hipSuccess) {
    (void)hipGetLastError();
    delete J;
    set_error("could not load the compiled physics module");
    return LDG_EDEVICE;
  }
  for (int i = 0; i < 4; ++i) {
    if (hipModuleGetFunction(&J->grad[i / 2][i % 2], J->mod, low[i].c_str()) != hipSuccess ||
        hipModuleGetFunction(&J->resid[i / 2][i % 2], J->mod, low[4 + i].c_str()) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipModuleUnload(J->mod);
      delete J;
      set_error("compiled physics module lacks an operator kernel");
      return LDG_EDEVICE;
    }
  }
  {
    hipDeviceptr_t pnw = nullptr, pna = nullptr;
    size_t bytes = 0, bytes_a = 0;
    int naux_max = 0;
    if (hipModuleGetFunction(&J->ode, J->mod, "ldg_k_ode_stage") != hipSuccess ||
        hipModuleGetGlobal(&pnw, &bytes, J->mod, "ldg_user_nw") != hipSuccess || bytes != sizeof(int) ||
        hipMemcpyDtoH(&J->nw, pnw, sizeof(int)) != hipSuccess ||
        hipModuleGetGlobal(&pna, &bytes_a, J->mod, "ldg_user_naux") != hipSuccess || bytes_a != sizeof(int) ||
        hipMemcpyDtoH(&naux_max, pna, sizeof(int)) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipModuleUnload(J->mod);
      delete J;
      set_error("compiled physics module lacks the ODE kernel or its sizes");
      return LDG_EDEVICE;
    }
    if (md.naux > naux_max) {
      (void)hipModuleUnload(J->mod);
      delete J;
      set_error("desc->naux = " + std::to_string(md.naux) + " exceeds LdgUser::NAUX = " + std::to_string(naux_max) +
                " (the kernels hold NAUX aux values per point)");
      return LDG_EINVAL;
    }
  }
  for (int f = 0; f < 2; ++f) {
    const int rsz = f ? 4 : 8;
    J->epb_grad[f] = pick_epb_n(m.nn, grad_bytes(md.ncu, m.nd, m.p1, rsz));
    for (int t = 0; t < 2; ++t)
      J->epb_resid[f][t] = pick_epb_n(m.nn, resid_bytes(md.ncu, md.hasq, t ? 2 : 1, m.nd, m.p1, rsz));
  }
  md.jit = J;
  return LDG_OK;
}

void jit_release(Model& md) {
  if (!md.jit) return;
  (void)hipModuleUnload(md.jit->mod);
  delete md.jit;
  md.jit = nullptr;
}

ldg_status jit_check(const char* user, int nd, int p1, int ncu, bool hasq) {
  return compile(user, nd, p1, false, ncu, hasq, nullptr, nullptr);
}

namespace {
ldg_status launch(hipFunction_t f, int64_t E, int epb, int nn, void** args, hipStream_t s) {
  const unsigned nblk = (unsigned)((E + epb - 1) / epb);
  if (nblk == 0) return LDG_OK;
  if (hipModuleLaunchKernel(f, nblk, 1, 1, (unsigned)(epb * nn), 1, 1, 0, s, args, nullptr) != hipSuccess) {
    set_error(std::string("launch of a compiled physics kernel failed: ") + hipGetErrorString(hipGetLastError()));
    return LDG_EDEVICE;
  }
  return LDG_OK;
}
}  // namespace

// same argument lists as the built-in instances (see launch_grad / launch_resid)
ldg_status jit_grad(const Model& md, const double* u, void* q, bool fp32, bool with_data, hipStream_t s) {
  if (!md.hasq) return LDG_OK;
  const Mesh& m = *md.mesh;
  MeshDev mdv = m.dev_op(0);
  ModelDev mod = md.dev();
  const double* qoff = nullptr;
  const float* dux = nullptr;
  BasisTab tab = m.tab;
  BasisTabF tabf = m.tabf;
  void* args[] = {&mdv, fp32 ? (void*)&tabf : (void*)&tab, &mod, (void*)&u, &q, (void*)&qoff, (void*)&dux};
  return launch(md.jit->grad[fp32][with_data], m.op_E(0), md.jit->epb_grad[fp32], m.nn, args, s);
}

ldg_status jit_resid(const Model& md, const TimeDev& t, const double* u, const void* q, const double* v,
                     const void* dq, double* out, bool fp32, bool tangent, hipStream_t s) {
  const Mesh& m = *md.mesh;
  MeshDev mdv = m.dev_op(1);
  ModelDev mod = md.dev();
  TimeDev td = t;
  BasisTab tab = m.tab;
  BasisTabF tabf = m.tabf;
  const double* dterm = nullptr;
  float* Fout = nullptr;
  void* args[] = {&mdv,     fp32 ? (void*)&tabf : (void*)&tab, &mod, &td, (void*)&u, (void*)&q, (void*)&v,
                  (void*)&dq, (void*)&dterm, &out, &Fout};
  return launch(md.jit->resid[fp32][tangent], m.op_E(1), md.jit->epb_resid[fp32][tangent], m.nn, args, s);
}

int jit_ode_size(const Model& md) { return md.jit ? md.jit->nw : 0; }

ldg_status jit_ode(const Model& md, const TimeDev& t, double alpha, double beta, const double* u, double* w,
                   hipStream_t s) {
  const Mesh& m = *md.mesh;
  int64_t nodes = m.E * (int64_t)m.nn;
  int nn = m.nn;
  ModelDev mod = md.dev();
  double a0 = t.a0, c1 = t.c1, c2 = t.c2;
  const double* r1 = t.r1;
  const double* r2 = t.r2;
  void* args[] = {&nodes, &nn, &mod, &alpha, &beta, &a0, &c1, (void*)&r1, &c2, (void*)&r2, (void*)&u, &w};
  const unsigned nblk = (unsigned)((nodes + 255) / 256);
  if (nblk == 0) return LDG_OK;
  if (hipModuleLaunchKernel(md.jit->ode, nblk, 1, 1, 256, 1, 1, 0, s, args, nullptr) != hipSuccess) {
    set_error(std::string("launch of the ODE kernel failed: ") + hipGetErrorString(hipGetLastError()));
    return LDG_EDEVICE;
  }
  return LDG_OK;
}

}  // namespace ldg
