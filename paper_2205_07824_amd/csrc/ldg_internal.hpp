// Internal definitions shared by the host code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ldg.h"

namespace ldg {

constexpr int MAXP1 = 6;        // p <= 5
constexpr int MAXTAG = 8;
constexpr int MAXMU = 8;

__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// 1D tables on the p+1 Gauss-Legendre nodes, passed to kernels by value.
struct BasisTab {
  double x[MAXP1];            // nodes (ascending)
  double w[MAXP1];            // Gauss-Legendre weights
  double D[MAXP1][MAXP1];     // D[a][m] = l_m'(x_a)
  double lf[2][MAXP1];        // lf[s][m] = l_m(-1) for s = 0, l_m(+1) for s = 1
};
struct BasisTabF {            // single-precision copy
  float x[MAXP1], w[MAXP1], D[MAXP1][MAXP1], lf[2][MAXP1];
};

// Device view of a mesh.
struct MeshDev {
  int E;
  int nbf;
  const double* coef;    // [E][2^nd][nd] multilinear monomial coefficients: x(xi) = sum_m coef[m] prod_{k in m} xi_k
  const int32_t* nbr;    // [E][2nd] >= 0 neighbour element; < 0: -(1 + boundary face index)
  const int32_t* btag;   // [nbf] boundary tag
  const int32_t* order;  // [E] element visit order of the operator kernels (a permutation of 0..E-1)
};

// Device view of a model's parameters.
struct ModelDev {
  double mu[MAXMU];
  int naux;
  const double* aux;     // [E][naux][nn]
  const double* src;     // nonlinear models: [E][ncu][nn] source at the (collocated) nodes
  const double* bdata;   // nonlinear models: [nbf][ncu][nfp]
  int bc_kind[MAXTAG];
  int nbc;
};

// time wrapper coefficients
struct TimeDev {
  double a0, c1, c2;
  const double* r1;
  const double* r2;
};

// --------------------------------------------------------------------------
// Forward-mode dual number used by the nonlinear tangent kernels.
// Non-smooth points: |x|' = sign(x) with sign(0) = +1; max(a,b)' = a' if a >= b.
// --------------------------------------------------------------------------
template <class R>
struct Dl {
  R v, d;
};
template <class R> __host__ __device__ inline Dl<R> operator+(Dl<R> a, Dl<R> b) { return {a.v + b.v, a.d + b.d}; }
template <class R> __host__ __device__ inline Dl<R> operator-(Dl<R> a, Dl<R> b) { return {a.v - b.v, a.d - b.d}; }
template <class R> __host__ __device__ inline Dl<R> operator-(Dl<R> a) { return {-a.v, -a.d}; }
template <class R> __host__ __device__ inline Dl<R> operator*(Dl<R> a, Dl<R> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class R> __host__ __device__ inline Dl<R> operator*(R a, Dl<R> b) { return {a * b.v, a * b.d}; }
template <class R> __host__ __device__ inline Dl<R> operator*(Dl<R> a, R b) { return {a.v * b, a.d * b}; }
template <class R> __host__ __device__ inline Dl<R> operator+(Dl<R> a, R b) { return {a.v + b, a.d}; }
template <class R> __host__ __device__ inline Dl<R> operator+(R a, Dl<R> b) { return {a + b.v, b.d}; }
template <class R> __host__ __device__ inline Dl<R> operator-(Dl<R> a, R b) { return {a.v - b, a.d}; }
template <class R> __host__ __device__ inline Dl<R> operator-(R a, Dl<R> b) { return {a - b.v, -b.d}; }
template <class R> __host__ __device__ inline Dl<R> operator/(Dl<R> a, Dl<R> b) {
  R inv = R(1) / b.v;
  R q = a.v * inv;
  return {q, (a.d - q * b.d) * inv};
}
template <class R> __host__ __device__ inline Dl<R> operator/(Dl<R> a, R b) { R inv = R(1) / b; return {a.v * inv, a.d * inv}; }
template <class R> __host__ __device__ inline Dl<R>& operator+=(Dl<R>& a, Dl<R> b) { a = a + b; return a; }
template <class R> __host__ __device__ inline Dl<R>& operator-=(Dl<R>& a, Dl<R> b) { a = a - b; return a; }

// value-type traits: R (plain) or Dl<R>
template <class V> struct VT;
template <> struct VT<double> {
  using R = double;
  __host__ __device__ static double mk(double x, double = 0) { return x; }
  __host__ __device__ static double val(double x) { return x; }
  __host__ __device__ static double tan(double) { return 0; }
};
template <> struct VT<float> {
  using R = float;
  __host__ __device__ static float mk(float x, float = 0) { return x; }
  __host__ __device__ static float val(float x) { return x; }
  __host__ __device__ static float tan(float) { return 0; }
};
template <class R> struct VT<Dl<R>> {
  using Rr = R;
  __host__ __device__ static Dl<R> mk(R x, R d = 0) { return {x, d}; }
  __host__ __device__ static R val(Dl<R> x) { return x.v; }
  __host__ __device__ static R tan(Dl<R> x) { return x.d; }
};

__device__ inline double vsqrt(double x) { return sqrt(x); }
__device__ inline float vsqrt(float x) { return sqrtf(x); }
template <class R> __device__ inline Dl<R> vsqrt(Dl<R> a) { R s = vsqrt(a.v); return {s, a.d / (R(2) * s)}; }
__device__ inline double vabs(double x) { return x >= 0 ? x : -x; }
__device__ inline float vabs(float x) { return x >= 0 ? x : -x; }
template <class R> __device__ inline Dl<R> vabs(Dl<R> a) { return a.v >= 0 ? a : -a; }
__device__ inline double vmax(double a, double b) { return a >= b ? a : b; }
__device__ inline float vmax(float a, float b) { return a >= b ? a : b; }
template <class R> __device__ inline Dl<R> vmax(Dl<R> a, Dl<R> b) { return a.v >= b.v ? a : b; }

// --------------------------------------------------------------------------
// Geometry: Jacobian of the multilinear map from its monomial coefficients.
// J[i][j] = d x_i / d xi_j.
// --------------------------------------------------------------------------
template <int D, class R>
__device__ inline void jacobian_at(const double* __restrict__ c /*[2^D][D]*/, const R* xi, R J[D][D]) {
#pragma unroll
  for (int j = 0; j < D; ++j) {
#pragma unroll
    for (int i = 0; i < D; ++i) J[i][j] = R(0);
#pragma unroll
    for (int m = 0; m < (1 << D); ++m) {
      if (!((m >> j) & 1)) continue;
      R t = R(1);
#pragma unroll
      for (int k = 0; k < D; ++k)
        if (k != j && ((m >> k) & 1)) t *= xi[k];
#pragma unroll
      for (int i = 0; i < D; ++i) J[i][j] += R(c[m * D + i]) * t;
    }
  }
}

// adj[j][k] = det(J) * (J^-1)[j][k]; returns det(J)
template <int D, class R>
__device__ inline R adjugate(const R J[D][D], R adj[D][D]) {
  if constexpr (D == 2) {
    adj[0][0] = J[1][1]; adj[0][1] = -J[0][1];
    adj[1][0] = -J[1][0]; adj[1][1] = J[0][0];
    return J[0][0] * J[1][1] - J[0][1] * J[1][0];
  } else {
    // columns a = J[.][0], b = J[.][1], c = J[.][2]; rows of adj are b x c, c x a, a x b
    adj[0][0] = J[1][1] * J[2][2] - J[2][1] * J[1][2];
    adj[0][1] = J[2][1] * J[0][2] - J[0][1] * J[2][2];
    adj[0][2] = J[0][1] * J[1][2] - J[1][1] * J[0][2];
    adj[1][0] = J[1][2] * J[2][0] - J[2][2] * J[1][0];
    adj[1][1] = J[2][2] * J[0][0] - J[0][2] * J[2][0];
    adj[1][2] = J[0][2] * J[1][0] - J[1][2] * J[0][0];
    adj[2][0] = J[1][0] * J[2][1] - J[2][0] * J[1][1];
    adj[2][1] = J[2][0] * J[0][1] - J[0][0] * J[2][1];
    adj[2][2] = J[0][0] * J[1][1] - J[1][0] * J[0][1];
    return J[0][0] * adj[0][0] + J[1][0] * adj[0][1] + J[2][0] * adj[0][2];
  }
}

// Scaled outward normal N = ds * n on face (dir, side): (2 side - 1) * row dir of adj(J).
// (Nanson: n ds = det(J) J^-T N_ref dA_ref.)
template <int D, class R>
__device__ inline void scaled_normal(const R J[D][D], int dir, int side, R N[D]) {
  R adj[D][D];
  (void)adjugate<D, R>(J, adj);
  R s = side ? R(1) : R(-1);
#pragma unroll
  for (int k = 0; k < D; ++k) N[k] = s * adj[dir][k];
}

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
  MeshDev dev() const { return MeshDev{(int)E, (int)nbf, d_coef, d_nbr, d_btag, d_order}; }
};

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

// operator entry points (ldg_operator.hip)
ldg_status op_grad(const Model& md, const double* u, void* q, bool fp32, bool with_data, hipStream_t s);
ldg_status op_resid(const Model& md, const TimeDev& t, const double* u, const void* q, double* out, bool fp32,
                    bool with_data, hipStream_t s);
ldg_status op_jvp_nonlinear(const Model& md, const TimeDev& t, const double* u, const void* q, const double* v,
                            const void* dq, double* out, bool fp32, hipStream_t s);
ldg_status op_data_terms(Model& md, hipStream_t s);
ldg_status op_mfma_jvp(const Model& md, const TimeDev& t, const double* v, double* out, bool fp16, hipStream_t s);
void mfma_release(const Model& md);

// shared host helpers (ldg_api.hip)
TimeDev make_time(const ldg_time* t, bool with_rhs);
ldg_status residual_impl(Model& md, const ldg_time* t, const double* u, double* G, double* q_out, bool fp32,
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
