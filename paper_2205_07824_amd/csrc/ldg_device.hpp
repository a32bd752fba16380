// Definitions shared by the gfx950 kernels and the host code: limits, the device
// views of mesh, model and time wrapper, the forward-mode dual number, and the
// pointwise geometry helpers.  Device-only (no host library types), so that the
// runtime compiler can build it together with user physics.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#else
#include <type_traits>
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif

namespace ldg {

// boundary condition kinds, the values of the ABI's ldg_bc_kind
enum BcKind { BC_DIRICHLET = 0, BC_NEUMANN = 1, BC_EXTRAP = 2 };

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
  // batched products (block probing): work-group row blockIdx.y works on the
  // y-th of gridDim.y products, whose per-product vectors (direction, tangent of
  // q, result) lie bsn and bsq elements apart; 0 for a single product
  int64_t bsn = 0, bsq = 0;
};

// Device view of a model's parameters.
// void for any well-formed type list (member detection in the run-time compiled physics)
template <class... T>
struct VoidOf { using type = void; };

struct ModelDev {
  double mu[MAXMU];
  int naux;
  const double* aux;     // [E][naux][nn]
  const double* src;     // nonlinear models: [E][ncu][nn] source at the (collocated) nodes
  const double* bdata;   // nonlinear models: [nbf][ncu][nfp]
  int bc_kind[MAXTAG];
  int nbc;
  // face traces of the linearization point (u, q(u)) for the FP64 tangent kernels,
  // [E][2 nd][(p+1)^(nd-1)][ncu (1 + nd)] (u, then q in [c][k] order); nullptr = none
  const double* tr;
  const float* tr32;   // the same for the FP32 tangent kernels (FP32 linearization point cache)
  double* trt;         // face traces of the product's direction (v, tangent of q), FP64
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

}  // namespace ldg
