// LDG operator kernels for gfx950 (instantiated per model kind in ldg_op_*.hip): the local gradient q (Eq. 1a in weak form),
// the residual R(u) with the implicit time wrapper, and its exact tangent.
//
// Layout: one thread per (element, node); EPB elements per work-group.  The
// basis is the Lagrange basis on the (p+1)^D Gauss-Legendre nodes and the
// quadrature is collocated with the nodes, so the element mass matrix is
// diagonal (w_i |J_i|) and every volume contraction is a sum-factorized
// application of the 1D derivative matrix along one direction (p+1 products
// per node and direction), staged through LDS.
//
// Faces are handled element-centrically: every element evaluates the numerical
// flux on each of its 2D faces from its own trace and the neighbour's trace
// (read directly from the neighbour's nodal lines), and lifts it into its own
// nodes.  No element writes another element's output, so there are no atomics,
// no face colouring passes, and the result is bitwise deterministic.
//
// Face work is organised by reference direction (a compile-time constant), so
// the line strides, the tangential directions and the normal (cross product of
// the two tangential Jacobian columns) need no per-lane selects.  The 1D tables
// live in LDS.  Work-groups take elements in the mesh's visit order (the
// Morton order of the element centroids), and each of the eight XCDs (which
// receive work-groups round-robin) walks a contiguous range of that order, so
// that most face neighbours are in flight on the same XCD and hit its L2.
#pragma once

#include "ldg_physics.hpp"

namespace ldg {

// FP64 1/sqrt(x) and 1/x from the hardware estimates refined by two Newton
// steps: fewer issue slots than the correctly rounded sequences, within a few
// ulp (the FP32 kernels keep the plain operations, measured faster there).
__device__ inline double fast_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}
__device__ inline double fast_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}

template <class R> struct TabOf;
template <> struct TabOf<double> { using T = BasisTab; };
template <> struct TabOf<float> { using T = BasisTabF; };

// Elements per work-group: fill 256 threads (2D) or 128 threads (3D elements,
// where fewer waves per barrier measured faster), bounded by an LDS budget.
// Plain constexpr functions of the sizes, so that the launcher of kernels
// compiled at run time computes the same numbers.
__host__ __device__ constexpr int pick_epb_n(int nn, int bytes_per_elem) {
  int e = (nn >= 27 ? 128 : 256) / nn;
  if (e < 1) e = 1;
  while (e > 1 && e * bytes_per_elem > 40 * 1024) --e;
  return e;
}
template <int NN, int BYTES_PER_ELEM>
constexpr int pick_epb() { return pick_epb_n(NN, BYTES_PER_ELEM); }

__host__ __device__ constexpr int geo_tab_size(int d, int p1) {
  return (d * ipow(p1, d - 1) + ((d == 3) ? 2 * d * 2 * p1 : 2 * d)) * d;
}
// LDS bytes per element of the gradient and residual kernels (rsz = sizeof(R))
__host__ __device__ constexpr int grad_bytes(int ncu, int d, int p1, int rsz) {
  return rsz * (ncu * ipow(p1, d) + 2 * d * ncu * d * ipow(p1, d - 1) + geo_tab_size(d, p1)) + 8 * (1 << d) * d;
}
// (the tangent kernel, mode 2, reads q and its tangent from global memory and
// stages only the dual state u in LDS)
__host__ __device__ constexpr int resid_bytes(int ncu, bool hasq, int mode, int d, int p1, int rsz) {
  return (mode == 2 ? 2 * rsz * ncu * ipow(p1, d) : rsz * (ncu * ipow(p1, d) + (hasq ? ncu * d * ipow(p1, d) : 0))) +
         rsz * (ncu * d * ipow(p1, d) + 2 * d * ncu * ipow(p1, d - 1) + geo_tab_size(d, p1)) + 8 * (1 << d) * d;
}

template <int P1>
struct TabLayout {
  static constexpr int X = 0, W = P1, DM = 2 * P1, LF = 2 * P1 + P1 * P1, SIZE = 4 * P1 + P1 * P1;
};

// copy the 1D tables into LDS: x, w, D (row-major D[a][m]), lf[0], lf[1]
template <int P1, class R, class TAB>
__device__ inline void stage_tables(const TAB& tab, R* st) {
  using L = TabLayout<P1>;
  for (int t = threadIdx.x; t < L::SIZE; t += blockDim.x) {
    R v;
    if (t < L::W) v = tab.x[t];
    else if (t < L::DM) v = tab.w[t - L::W];
    else if (t < L::LF) { const int r = (t - L::DM) / P1, c = (t - L::DM) % P1; v = tab.D[r][c]; }
    else { const int r = (t - L::LF) / P1, c = (t - L::LF) % P1; v = tab.lf[r][c]; }
    st[t] = v;
  }
}

// work-group -> block of slots in the mesh's element visit order, XCD-aware
// (work-group b runs on XCD b % 8, and each XCD walks a contiguous range)
__device__ inline int64_t xcd_block(int64_t b, int64_t nblk) {
  const int64_t q = nblk >> 3;
  if (b < (q << 3)) return (b & 7) * q + (b >> 3);
  return b;
}

__host__ __device__ constexpr int stride_c(int P1, int k) { return k == 0 ? 1 : (k == 1 ? P1 : P1 * P1); }

// tangential directions of a face normal to DIR
template <int D, int DIR> struct Tang {
  static constexpr int T0 = (DIR == 0) ? 1 : 0;
  static constexpr int T1 = (D == 3) ? ((DIR == 2) ? 1 : 2) : -1;
};

// column j of the Jacobian of the multilinear map at xi
template <int D, int J, class R, bool AFF = false>
__device__ inline void jac_col(const double* __restrict__ c, const R* xi, R* col) {
  if constexpr (AFF) {
    // affine element: only the linear monomial of the map contributes
#pragma unroll
    for (int i = 0; i < D; ++i) col[i] = R(c[(1 << J) * D + i]);
    return;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) col[i] = R(0);
#pragma unroll
  for (int m = 0; m < (1 << D); ++m) {
    if (!((m >> J) & 1)) continue;
    R t = R(1);
#pragma unroll
    for (int k = 0; k < D; ++k)
      if (k != J && ((m >> k) & 1)) t *= xi[k];
#pragma unroll
    for (int i = 0; i < D; ++i) col[i] += R(c[m * D + i]) * t;
  }
}

// scaled outward normal N = ds n at a point of face (DIR, side): (2 side - 1) * row DIR of adj(J)
template <int D, int DIR, class R, bool AFF = false>
__device__ inline void face_normal(const double* __restrict__ c, const R* xi, int side, R* N) {
  const R s = side ? R(1) : R(-1);
  if constexpr (D == 2) {
    constexpr int T = 1 - DIR;
    R col[2];
    jac_col<2, T, R, AFF>(c, xi, col);
    if constexpr (DIR == 0) { N[0] = s * col[1]; N[1] = -s * col[0]; }
    else { N[0] = -s * col[1]; N[1] = s * col[0]; }
  } else {
    // row DIR of adj = col(DIR+1) x col(DIR+2) (cyclic)
    constexpr int A = (DIR + 1) % 3, B = (DIR + 2) % 3;
    R a[3], b[3];
    jac_col<3, A, R, AFF>(c, xi, a);
    jac_col<3, B, R, AFF>(c, xi, b);
    N[0] = s * (a[1] * b[2] - a[2] * b[1]);
    N[1] = s * (a[2] * b[0] - a[0] * b[2]);
    N[2] = s * (a[0] * b[1] - a[1] * b[0]);
  }
}

// full Jacobian J[i][j] = d x_i / d xi_j from its columns
template <int D, class R, bool AFF>
__device__ inline void jac_full(const double* __restrict__ c, const R* xi, R J[D][D]) {
  R col[D];
  jac_col<D, 0, R, AFF>(c, xi, col);
#pragma unroll
  for (int i = 0; i < D; ++i) J[i][0] = col[i];
  jac_col<D, 1, R, AFF>(c, xi, col);
#pragma unroll
  for (int i = 0; i < D; ++i) J[i][1] = col[i];
  if constexpr (D == 3) {
    jac_col<D, 2, R, AFF>(c, xi, col);
#pragma unroll
    for (int i = 0; i < D; ++i) J[i][2] = col[i];
  }
}

template <int D, int P1>
__device__ inline void node_index(int i, int* a) {
#pragma unroll
  for (int k = 0; k < D; ++k) { a[k] = i % P1; i /= P1; }
}

// tangential flat index of node a[] on a face normal to dir (lower tangential direction fastest)
template <int D, int P1>
__device__ inline int face_index_of_node(const int* a, int dir) {
  int f = 0, s = 1;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (k == dir) continue;
    f += a[k] * s;
    s *= P1;
  }
  return f;
}

template <int D, int P1>
struct GeoTab {
  static constexpr int NFP = ipow(P1, D - 1), NF = 2 * D;
  static constexpr int NVC = D * NFP;                       // volume columns
  static constexpr int NFC = (D == 3) ? NF * 2 * P1 : NF;   // face columns
  static constexpr int NCOL = NVC + NFC;
  static constexpr int SIZE = NCOL * D;
};

// Column tables of one element, evaluated by its nl lanes:
//   entry t < NVC:  column j = t / NFP at the tangential tuple t % NFP (lower direction fastest)
//   3D face column (F, h, idx): h = 0 column A = (dir+1)%3 with xi_B = x[idx],
//                               h = 1 column B = (dir+2)%3 with xi_A = x[idx], xi_dir = -1/+1
//   2D face column F: column 1-dir at xi_dir = -1/+1 (constant along the edge)
// A column j is bilinear (3D) or linear (2D) in the other coordinates, taken in
// increasing direction order (va, vb); the code is the same for every lane.
template <int D, int P1, class R>
__device__ inline void build_geo(const double* c, const R* tx, R* g, int lane, int nl) {
  using G = GeoTab<D, P1>;
  for (int t = lane; t < G::NCOL; t += nl) {
    int j;
    R va;
    if constexpr (D == 3) {
      R vb;
      if (t < G::NVC) {
        j = t / G::NFP;
        const int r = t % G::NFP;
        va = tx[r % P1];
        vb = tx[r / P1];
      } else {
        const int uu = t - G::NVC;
        const int F = uu / (2 * P1), h = (uu / P1) & 1, idx = uu % P1;
        const int dir = F >> 1;
        const int A = (dir + 1) % 3, B = (dir + 2) % 3;
        const R sd = (F & 1) ? R(1) : R(-1);
        j = h ? B : A;
        const int other = h ? A : B;
        if (dir < other) { va = sd; vb = tx[idx]; } else { va = tx[idx]; vb = sd; }
      }
      const int o0 = (j == 0) ? 1 : 0, o1 = (j == 2) ? 1 : 2;
      const int m0 = 1 << j, m1 = m0 | (1 << o0), m2 = m0 | (1 << o1), m3 = m1 | (1 << o1);
      const R vab = va * vb;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        g[t * 3 + k] = R(c[m0 * 3 + k]) + R(c[m1 * 3 + k]) * va + R(c[m2 * 3 + k]) * vb + R(c[m3 * 3 + k]) * vab;
    } else {
      if (t < G::NVC) {
        j = t / P1;
        va = tx[t % P1];
      } else {
        const int F = t - G::NVC;
        j = 1 - (F >> 1);
        va = (F & 1) ? R(1) : R(-1);
      }
      const int m0 = 1 << j, m1 = m0 | (1 << (1 - j));
#pragma unroll
      for (int k = 0; k < 2; ++k) g[t * 2 + k] = R(c[m0 * 2 + k]) + R(c[m1 * 2 + k]) * va;
    }
  }
}

// Jacobian at node a[] from the tables (or the constant columns of an affine map)
template <int D, int P1, class R, bool AFF>
__device__ inline void geo_jac(const R* g, const double* __restrict__ c, const int* a, R J[D][D]) {
  if constexpr (AFF) {
    R xi0[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xi0[k] = R(0);
    jac_full<D, R, true>(c, xi0, J);
  } else {
    constexpr int NFP = GeoTab<D, P1>::NFP;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const R* col = g + (j * NFP + face_index_of_node<D, P1>(a, j)) * D;
#pragma unroll
      for (int k = 0; k < D; ++k) J[k][j] = col[k];
    }
  }
}

// scaled outward normal N = ds n at face point (t0, t1) of face (DIR, side)
template <int D, int P1, int DIR, class R, bool AFF>
__device__ inline void geo_normal(const R* g, const double* __restrict__ c, int side, int t0, int t1, R* N) {
  if constexpr (AFF) {
    R xi0[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xi0[k] = R(0);
    face_normal<D, DIR, R, true>(c, xi0, side, N);
  } else {
    using G = GeoTab<D, P1>;
    const int F = 2 * DIR + side;
    const R s = side ? R(1) : R(-1);
    if constexpr (D == 2) {
      const R* col = g + (G::NVC + F) * 2;
      if constexpr (DIR == 0) { N[0] = s * col[1]; N[1] = -s * col[0]; }
      else { N[0] = -s * col[1]; N[1] = s * col[0]; }
    } else {
      constexpr int A = (DIR + 1) % 3, B = (DIR + 2) % 3;
      constexpr int T0 = Tang<3, DIR>::T0;
      const int iB = (B == T0) ? t0 : t1;
      const int iA = (A == T0) ? t0 : t1;
      const R* a = g + (G::NVC + (F * 2 + 0) * P1 + iB) * 3;
      const R* b = g + (G::NVC + (F * 2 + 1) * P1 + iA) * 3;
      N[0] = s * (a[1] * b[2] - a[2] * b[1]);
      N[1] = s * (a[2] * b[0] - a[0] * b[2]);
      N[2] = s * (a[0] * b[1] - a[1] * b[0]);
    }
  }
}

template <int KIND, int D, int P1, class R>
struct GradCfg {
  static constexpr int NCU = Phys<KIND, D>::NCU, NN = ipow(P1, D), NFP = ipow(P1, D - 1), NF = 2 * D, NV = 1 << D;
  static constexpr int BYTES = sizeof(R) * (NCU * NN + NF * NCU * D * NFP + GeoTab<D, P1>::SIZE) + 8 * NV * D;
  static_assert(BYTES == grad_bytes(NCU, D, P1, sizeof(R)), "one formula for the host and the kernels");
  static constexpr int EPB = pick_epb<NN, BYTES>();
};

// the trace arrays of a precision (FP64 or FP32)
template <class R> __device__ inline const R* lin_traces(const ModelDev& md) {
  if constexpr (std::is_same<R, double>::value) return md.tr; else return md.tr32;
}
template <class R> __device__ inline R* dir_traces(const ModelDev& md) {
  static_assert(std::is_same<R, double>::value, "direction traces are FP64");
  return md.trt;
}

// Face traces of a linearization point for the tangent kernels: for every
// element, face F = 2 DIR + side and face point ff (the numbering of k_resid's
// faces), u and q(u) extrapolated to the face along the lines normal to it, in
// the same order of operations as k_resid's own extrapolation, stored
// [E][NF][NCU (1 + D)][NFP] (u, then q in [c][k] order).  Formed once per
// linearization point; the tangent kernel then reads a neighbour's NCU (1 + D)
// trace values at a face point instead of its P1-node lines of u and q.  The
// FP64 tangent can also read the same traces of the product's direction (v and
// the tangent of q), written by k_grad<..., TRT> as it forms the tangent of q.
template <int D, int P1, int NCU, class R = double, class S = double>
__global__ void __launch_bounds__(256) k_face_traces(int64_t E, typename TabOf<R>::T tab, const S* __restrict__ u,
                                                     const R* __restrict__ q, R* __restrict__ tr) {
  constexpr int NN = ipow(P1, D), NF = 2 * D, NFP = ipow(P1, D - 1), NVT = NCU * (1 + D);
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E * NF * NFP) return;
  const int ff = (int)(t % NFP);
  const int F = (int)((t / NFP) % NF);
  const int64_t K = t / (NF * NFP);
  const int dir = F >> 1, side = F & 1;
  const int T0 = dir == 0 ? 1 : 0;
  const int T1 = D == 3 ? (dir == 2 ? 1 : 2) : 0;
  const int t0 = ff % P1, t1 = D == 3 ? ff / P1 : 0;
  int base = t0 * stride_c(P1, T0);
  if (D == 3) base += t1 * stride_c(P1, T1);
  const int SD = stride_c(P1, dir);
  const R* l = tab.lf[side];
  R* o = tr + (K * NF + F) * NVT * NFP + ff;
#pragma unroll
  for (int c = 0; c < NCU; ++c) {
    const S* up = u + (K * NCU + c) * NN + base;
    R a = R(0);
#pragma unroll
    for (int mm = 0; mm < P1; ++mm) a += l[mm] * R(up[mm * SD]);
    o[c * NFP] = a;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const R* qp = q + ((K * NCU + c) * D + k) * NN + base;
      R b = R(0);
#pragma unroll
      for (int mm = 0; mm < P1; ++mm) b += l[mm] * qp[mm * SD];
      o[(NCU + c * D + k) * NFP] = b;
    }
  }
}

template <int KIND, int D, int P1, class R, int MODE>
struct ResidCfg {
  using PH = Phys<KIND, D>;
  using V = typename std::conditional<MODE == 2, Dl<R>, R>::type;
  static constexpr int NCU = PH::NCU, NN = ipow(P1, D), NFP = ipow(P1, D - 1), NF = 2 * D, NV = 1 << D;
  static constexpr bool HASQ = PH::HASQ;
  static constexpr int NQ = HASQ ? NCU * D : 1;
  // q staged in LDS: the residual kernels (modes 0, 1); the tangent kernel reads q, dq from global memory
  static constexpr bool QLDS = HASQ && MODE != 2;
  static constexpr int BYTES = sizeof(V) * (NCU * NN + (QLDS ? NCU * D * NN : 0)) +
                               sizeof(R) * (NCU * D * NN + NF * NCU * NFP + GeoTab<D, P1>::SIZE) + 8 * NV * D;
  static_assert(BYTES == resid_bytes(NCU, HASQ, MODE, D, P1, sizeof(R)), "one formula for the host and the kernels");
  static constexpr int EPB = pick_epb<NN, BYTES>();
  // the linear 3D FP64 instance needs 98 VGPRs unconstrained (4 waves per SIMD);
  // capping it at 96 for a fifth wave measured 6 us faster on the 32^3 p=3 JVP
  // (an occupancy hint of 3 or 4 waves on the dual Navier-Stokes tangent spilled
  // registers to scratch and measured 1.4-1.8x slower than the unconstrained 2)
  static constexpr int MIN_WAVES =
      (Phys<KIND, D>::LINEAR && D == 3 && MODE == 0 && std::is_same<R, double>::value) ? 5 : 1;
};

// ============================================================================
// Local gradient: q = M^-1 [ (u, div r) - <uhat n, r> ], evaluated in the
// equivalent strong form q = -grad u + M^-1 <(u- - uhat) n, r> (integration by
// parts is exact under the collocated Gauss rule for multilinear elements).
// DATA = true: Dirichlet uhat = g from bdata (nonlinear models); false:
// homogeneous (tangents, and linear models whose data enter through qoff).
// ============================================================================
// S: storage type of the state u (double; float for the FP32-state products)
// TRT: also write the face traces of u (here the product's direction) and of
// the q it forms to md.trt ([E][NF][NCU (1 + D)][NFP], as k_face_traces), the
// former from the face pass, the latter after staging q in the lifting buffer
template <int KIND, int D, int P1, class R, bool DATA, bool EXT = false, bool AFF = false, class S = double,
          bool TRT = false>
__global__ void __launch_bounds__(256)
k_grad(MeshDev m, typename TabOf<R>::T tab, ModelDev md, const S* __restrict__ u, R* __restrict__ q,
       const double* __restrict__ qoff, const float* __restrict__ dux = nullptr) {
  u += (int64_t)blockIdx.y * m.bsn;   // batched products (zero strides otherwise)
  q += (int64_t)blockIdx.y * m.bsq;
  using C = GradCfg<KIND, D, P1, R>;
  constexpr int NCU = C::NCU, NN = C::NN, NFP = C::NFP, NF = C::NF, NV = C::NV, EPB = C::EPB;
  using L = TabLayout<P1>;
  __shared__ R s_tab[L::SIZE];
  __shared__ R s_u[EPB][NCU][NN];
  __shared__ R s_L[EPB][NF][NCU][D][NFP];
  __shared__ double s_c[EPB][NV * D];
  __shared__ R s_g[EPB][AFF ? 1 : GeoTab<D, P1>::SIZE];
  __shared__ R s_lfw[2 * P1];

  __shared__ int s_K[EPB];
  const int64_t eb = xcd_block(blockIdx.x, gridDim.x);
  const int el = threadIdx.x / NN, i = threadIdx.x % NN;
  const bool active = eb * EPB + el < m.E;
  const int64_t K = active ? m.order[eb * EPB + el] : 0;
  if (threadIdx.x < EPB) s_K[threadIdx.x] = eb * EPB + threadIdx.x < m.E ? m.order[eb * EPB + threadIdx.x] : -1;
  stage_tables<P1, R>(tab, s_tab);
  if (active) {
#pragma unroll
    for (int c = 0; c < NCU; ++c) s_u[el][c][i] = R(u[(K * NCU + c) * NN + i]);
    for (int t = i; t < NV * D; t += NN) s_c[el][t] = m.coef[K * NV * D + t];
  }
  for (int t = threadIdx.x; t < 2 * P1; t += blockDim.x) s_lfw[t] = R(tab.lf[t / P1][t % P1] / tab.w[t % P1]);
  __syncthreads();
  const R* tx = s_tab + L::X;
  const R* tD = s_tab + L::DM;
  const R* tl = s_tab + L::LF;
  if constexpr (!AFF) {
    if (active) build_geo<D, P1, R>(s_c[el], tx, s_g[el], i, NN);
    __syncthreads();
  }

  // ---- faces, one reference direction at a time
  auto face_dir = [&](auto dirc, const int it) {
    constexpr int DIR = decltype(dirc)::value;
    constexpr int T0 = Tang<D, DIR>::T0, T1 = Tang<D, DIR>::T1;
    constexpr int SD = stride_c(P1, DIR);
    {
      const int e = it / (2 * NFP), side = (it / NFP) & 1, f = it % NFP;
      const int64_t Ke = s_K[e];
      if (Ke < 0) return;
      const int t0 = f % P1, t1 = (D == 3) ? f / P1 : 0;
      int base = t0 * stride_c(P1, T0);
      if constexpr (D == 3) base += t1 * stride_c(P1, T1);
      const R* l_own = tl + side * P1;
      const R* l_nbr = tl + (1 - side) * P1;
      R um[NCU], uh[NCU];
#pragma unroll
      for (int c = 0; c < NCU; ++c) {
        R sacc = R(0);
#pragma unroll
        for (int mm = 0; mm < P1; ++mm) sacc += l_own[mm] * s_u[e][c][base + mm * SD];
        um[c] = sacc;
      }
      const int F = 2 * DIR + side;
      const int nb = m.nbr[Ke * NF + F];
      if (nb >= 0) {
#pragma unroll
        for (int c = 0; c < NCU; ++c) {
          const S* un = u + ((int64_t)nb * NCU + c) * NN + base;
          R sacc = R(0);
#pragma unroll
          for (int mm = 0; mm < P1; ++mm) sacc += l_nbr[mm] * R(un[mm * SD]);
          uh[c] = R(0.5) * (um[c] + sacc);
        }
      } else {
        const int b = -(nb + 1);
        int tag = m.btag[b];
        tag = tag < 0 ? 0 : (tag >= md.nbc ? md.nbc - 1 : tag);
        const int kind = md.bc_kind[tag];
#pragma unroll
        for (int c = 0; c < NCU; ++c) {
          if (kind == BC_DIRICHLET)
            uh[c] = (DATA && md.bdata) ? R(md.bdata[((int64_t)b * NCU + c) * NFP + f]) : R(0);
          else
            uh[c] = um[c];
        }
      }
      R N[D];
      geo_normal<D, P1, DIR, R, AFF>(s_g[e], s_c[e], side, t0, t1, N);
#pragma unroll
      for (int c = 0; c < NCU; ++c)
#pragma unroll
        for (int k = 0; k < D; ++k) s_L[e][F][c][k][f] = (um[c] - uh[c]) * N[k];
      if constexpr (TRT) {
        R* o = dir_traces<R>(md) + (Ke * NF + F) * (NCU * (1 + D)) * NFP + f;
#pragma unroll
        for (int c = 0; c < NCU; ++c) o[c * NFP] = um[c];
      }
    }
  };
  // face items flattened over the directions (direction-major), so that the
  // direction is uniform across a wave whenever EPB * 2 * NFP is a multiple of 64
  for (int it = threadIdx.x; it < D * EPB * 2 * NFP; it += blockDim.x) {
    const int dir = it / (EPB * 2 * NFP), loc = it % (EPB * 2 * NFP);
    if (dir == 0) face_dir(std::integral_constant<int, 0>{}, loc);
    else if (dir == 1) face_dir(std::integral_constant<int, 1>{}, loc);
    else if constexpr (D == 3) face_dir(std::integral_constant<int, 2>{}, loc);
  }
  __syncthreads();
  if (!TRT && !active) return;
  R qreg[TRT ? NCU : 1][TRT ? D : 1];
  if (active) {

  int a[D];
  node_index<D, P1>(i, a);
  R J[D][D], adj[D][D];
  geo_jac<D, P1, R, AFF>(s_g[el], s_c[el], a, J);
  const R det = adjugate<D, R>(J, adj);
  const R idet = std::is_same<R, double>::value ? R(fast_rcp(double(det))) : R(1) / det;
  R liftw[NF];      // l_{a_dir}(side) / (w_{a_dir} det)
  int fidx[D];
#pragma unroll
  for (int F = 0; F < NF; ++F) liftw[F] = s_lfw[(F & 1) * P1 + a[F >> 1]] * idet;
#pragma unroll
  for (int dd = 0; dd < D; ++dd) fidx[dd] = face_index_of_node<D, P1>(a, dd);
#pragma unroll
  for (int c = 0; c < NCU; ++c) {
    R du[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if constexpr (EXT) {
        // reference gradient computed outside (MFMA GEMM)
        du[j] = R(dux[((K * NCU + c) * D + j) * NN + i]);
      } else {
        const int sj = stride_c(P1, j);
        const int b0 = i - a[j] * sj;
        const R* Drow = tD + a[j] * P1;
        R sacc = R(0);
#pragma unroll
        for (int mm = 0; mm < P1; ++mm) sacc += Drow[mm] * s_u[el][c][b0 + mm * sj];
        du[j] = sacc;
      }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
      R g = R(0);
#pragma unroll
      for (int j = 0; j < D; ++j) g += adj[j][k] * du[j];
      R qv = -g * idet;
#pragma unroll
      for (int F = 0; F < NF; ++F) qv += liftw[F] * s_L[el][F][c][k][fidx[F >> 1]];
      const int64_t o = ((K * NCU + c) * D + k) * NN + i;
      if (qoff) qv += R(qoff[o]);
      q[o] = qv;
      if constexpr (TRT) qreg[c][k] = qv;
    }
  }
  }  // active
  if constexpr (TRT) {
    // the element's q, staged in the lifting buffer (read completely above), extrapolated to its faces
    static_assert(NF * NFP >= NN, "the lifting buffer holds the element's q");
    __syncthreads();
    R* sq = &s_L[0][0][0][0][0];   // [EPB][NCU D][NN]
    if (active) {
#pragma unroll
      for (int c = 0; c < NCU; ++c)
#pragma unroll
        for (int k = 0; k < D; ++k) sq[(el * NCU * D + c * D + k) * NN + i] = qreg[c][k];
    }
    __syncthreads();
    for (int it = threadIdx.x; it < EPB * NF * NFP; it += blockDim.x) {
      const int e = it / (NF * NFP), F = (it / NFP) % NF, f = it % NFP;
      const int64_t Ke = s_K[e];
      if (Ke < 0) continue;
      const int dir = F >> 1, side = F & 1;
      const int T0 = dir == 0 ? 1 : 0;
      const int T1 = D == 3 ? (dir == 2 ? 1 : 2) : 0;
      const int t0 = f % P1, t1 = D == 3 ? f / P1 : 0;
      int base = t0 * stride_c(P1, T0);
      if (D == 3) base += t1 * stride_c(P1, T1);
      const int SD = stride_c(P1, dir);
      const R* l = tl + side * P1;
      R* o = dir_traces<R>(md) + (Ke * NF + F) * (NCU * (1 + D)) * NFP + f;
#pragma unroll
      for (int c = 0; c < NCU; ++c)
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const R* qp = sq + (e * NCU * D + c * D + k) * NN + base;
          R b = R(0);
#pragma unroll
          for (int mm = 0; mm < P1; ++mm) b += l[mm] * qp[mm * SD];
          o[(NCU + c * D + k) * NFP] = b;
        }
    }
  }
}

// ============================================================================
// Residual and tangent.
//   MODE 0: linear operator applied to the input (linear models' R_hom(u, q) and
//           their JVP), + a0 M u - M (c1 r1 + c2 r2) + dterm
//   MODE 1: nonlinear residual with data (source, Dirichlet/Neumann data) and
//           the time wrapper
//   MODE 2: tangent of the nonlinear residual at (u, q) in direction (v, dq),
//           dual-number arithmetic; + a0 M v
// ============================================================================
// S: storage type of the input vectors u, v (double; float for the FP32-state
// products of modes 0 and 2)
// TRC: read the face traces of the linearization point (u, q(u)); TRT (with
// TRC): also those of the direction (v, tangent of q) instead of its lines;
// PRB (with TRC, affine meshes): block probing, the neighbours' tangent-of-q
// traces in closed form (Mesh::probe_nbr)
template <int KIND, int D, int P1, class R, int MODE, bool EXT = false, bool AFF = false, class S = double,
          bool TRC = false, bool TRT = false, bool PRB = false>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(TRC ? 2 : ResidCfg<KIND, D, P1, R, MODE>::MIN_WAVES)))
k_resid(MeshDev m, typename TabOf<R>::T tab, ModelDev md, TimeDev tm, const S* __restrict__ u,
        const R* __restrict__ q, const S* __restrict__ v, const R* __restrict__ dq,
        const double* __restrict__ dterm, double* __restrict__ out, float* __restrict__ Fout = nullptr) {
  if (m.bsn) {   // batched products: the direction (tangent) or the argument (linear residual) and the result
    const int64_t by = blockIdx.y;
    if constexpr (MODE == 2) {
      v += by * m.bsn;
      if (dq) dq += by * m.bsq;
    } else {
      u += by * m.bsn;
      if (q) q += by * m.bsq;
    }
    out += by * m.bsn;
  }
  using C = ResidCfg<KIND, D, P1, R, MODE>;
  using V = typename C::V;
  using T = VT<V>;
  constexpr int NCU = C::NCU, NN = C::NN, NFP = C::NFP, NF = C::NF, NV = C::NV, EPB = C::EPB, NQ = C::NQ;
  constexpr bool HASQ = C::HASQ, QLDS = C::QLDS;
  constexpr int NA = Phys<KIND, D>::NAUX > 0 ? Phys<KIND, D>::NAUX : 1;
  using L = TabLayout<P1>;
  __shared__ R s_tab[L::SIZE];
  __shared__ V s_u[EPB][NCU][NN];
  __shared__ V s_q[EPB][QLDS ? NQ : 1][QLDS ? NN : 1];
  __shared__ R s_F[EPB][NCU][D][NN];
  __shared__ R s_Fh[EPB][NF][NCU][NFP];
  __shared__ double s_c[EPB][NV * D];
  __shared__ R s_g[EPB][AFF ? 1 : GeoTab<D, P1>::SIZE];

  __shared__ int s_K[EPB];
  const int64_t eb = xcd_block(blockIdx.x, gridDim.x);
  const int el = threadIdx.x / NN, i = threadIdx.x % NN;
  const bool active = eb * EPB + el < m.E;
  const int64_t K = active ? m.order[eb * EPB + el] : 0;
  if (threadIdx.x < EPB) s_K[threadIdx.x] = eb * EPB + threadIdx.x < m.E ? m.order[eb * EPB + threadIdx.x] : -1;
  stage_tables<P1, R>(tab, s_tab);
  // state loads: MODE 0 reads the input vector from u (the vector the linear
  // operator is applied to); MODE 2 pairs (u, v) and (q, dq).
  if (active) {
#pragma unroll
    for (int c = 0; c < NCU; ++c) {
      const int64_t o = (K * NCU + c) * NN + i;
      if constexpr (MODE == 2) s_u[el][c][i] = T::mk(R(u[o]), R(v[o]));
      else s_u[el][c][i] = R(u[o]);
    }
    if constexpr (QLDS) {
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const int64_t o = (K * NQ + c) * NN + i;
        s_q[el][c][i] = q[o];
      }
    }
    for (int t = i; t < NV * D; t += NN) s_c[el][t] = m.coef[K * NV * D + t];
  }
  __syncthreads();
  const R* tx = s_tab + L::X;
  const R* tw = s_tab + L::W;
  const R* tD = s_tab + L::DM;
  const R* tl = s_tab + L::LF;
  if constexpr (!AFF) {
    if (active) build_geo<D, P1, R>(s_c[el], tx, s_g[el], i, NN);
    __syncthreads();
  }

  // ---- faces: numerical flux times w ds, to LDS, one reference direction at a time
  auto face_dir = [&](auto dirc, const int it) {
    constexpr int DIR = decltype(dirc)::value;
    constexpr int T0 = Tang<D, DIR>::T0, T1 = Tang<D, DIR>::T1;
    constexpr int SD = stride_c(P1, DIR);
    {
      const int e = it / (2 * NFP), side = (it / NFP) & 1, ff = it % NFP;
      const int64_t Ke = s_K[e];
      if (Ke < 0) return;
      const int t0 = ff % P1, t1 = (D == 3) ? ff / P1 : 0;
      int base = t0 * stride_c(P1, T0);
      if constexpr (D == 3) base += t1 * stride_c(P1, T1);
      const R* l_own = tl + side * P1;
      const R* l_nbr = tl + (1 - side) * P1;
      V um[NCU], qm[NCU][D];
      R am[NA];
#pragma unroll
      for (int c = 0; c < NCU; ++c) {
        V sacc = T::mk(R(0));
#pragma unroll
        for (int mm = 0; mm < P1; ++mm) sacc += l_own[mm] * s_u[e][c][base + mm * SD];
        um[c] = sacc;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          V t = T::mk(R(0));
          if constexpr (QLDS) {
#pragma unroll
            for (int mm = 0; mm < P1; ++mm) t += l_own[mm] * s_q[e][c * D + k][base + mm * SD];
          } else if constexpr (HASQ) {
            // tangent kernel: the element's own q lines from global memory (cached);
            // with the traces formed (TRC), q(u) at the face point in one read, and
            // its tangent in one more (TRT: from the direction's traces) or from
            // the lines of the tangent
            const int64_t oq = ((Ke * NCU + c) * D + k) * NN + base;
            if constexpr (TRT) {
              const int64_t ot = ((Ke * NF + 2 * DIR + side) * (NCU * (1 + D)) + NCU + c * D + k) * NFP + ff;
              t = T::mk(lin_traces<R>(md)[ot], dir_traces<R>(md)[ot]);
            } else if constexpr (TRC) {
              R td = R(0);
#pragma unroll
              for (int mm = 0; mm < P1; ++mm) td += l_own[mm] * dq[oq + mm * SD];
              t = T::mk(lin_traces<R>(md)[((Ke * NF + 2 * DIR + side) * (NCU * (1 + D)) + NCU + c * D + k) * NFP + ff],
                        td);
            } else {
#pragma unroll
              for (int mm = 0; mm < P1; ++mm) t += l_own[mm] * T::mk(q[oq + mm * SD], dq[oq + mm * SD]);
            }
          }
          qm[c][k] = t;
        }
      }
#pragma unroll
      for (int t = 0; t < NA; ++t) {
        R sacc = R(0);
        if (t < md.naux) {
          const double* ap = md.aux + (Ke * md.naux + t) * NN + base;
#pragma unroll
          for (int mm = 0; mm < P1; ++mm) sacc += l_own[mm] * R(ap[mm * SD]);
        }
        am[t] = sacc;
      }
      R N[D], n[D];
      geo_normal<D, P1, DIR, R, AFF>(s_g[e], s_c[e], side, t0, t1, N);
      R nn2 = R(0);
#pragma unroll
      for (int k = 0; k < D; ++k) nn2 += N[k] * N[k];
      R ds, ids;
      if constexpr (std::is_same<R, double>::value) {
        ids = fast_rsqrt(nn2);
        ds = nn2 * ids;
      } else {
        ds = vsqrt(nn2);
        ids = R(1) / ds;
      }
#pragma unroll
      for (int k = 0; k < D; ++k) n[k] = N[k] * ids;
      R wf = tw[t0];
      if constexpr (D == 3) wf *= tw[t1];

      const int F = 2 * DIR + side;
      V Fh[NCU];
      const int nb = m.nbr[Ke * NF + F];
      if (nb >= 0) {
        // built-in models: this side's half of the flux first, then the neighbour's traces
        if constexpr (KIND != K_USER) half_normal_flux<KIND, D, V, R>(md.mu, md.naux, um, qm, am, n, Fh, false);
        V up[NCU], qp[NCU][D];
        R ap2[NA];
        // tangent with the traces of the linearization point formed (TRC): the
        // neighbour's u and q(u) at this face point (its face F ^ 1), one read per
        // value, consecutive face points adjacent ([E][NF][NCU (1 + D)][NFP]); TRT
        // also reads v and the tangent of q there from the direction's traces
        // block probing (PRB, affine meshes): the direction vanishes on the
        // neighbour and on its other neighbours (distance-2 colouring, distinct
        // neighbours), so the neighbour's tangent of q is the lifting of its jump
        // 0 - (0 + v)/2 on this face alone; its trace here is pfac v Nn, with Nn the
        // neighbour's face normal and pfac = -(1/2) sum_m l_m^2 / (w_m det)
        R pfac = R(0), Nn[D];
        if constexpr (MODE == 2 && HASQ && AFF && TRC && PRB) {
          {
            const double* cN = m.coef + (int64_t)nb * NV * D;
            R xi0[D], Jn[D][D], adjn[D][D];
#pragma unroll
            for (int k = 0; k < D; ++k) xi0[k] = R(0);
            face_normal<D, DIR, R, true>(cN, xi0, 1 - side, Nn);
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
              for (int j = 0; j < D; ++j) Jn[i][j] = R(cN[(1 << j) * D + i]);
            const R detn = adjugate<D, R>(Jn, adjn);
            R sl = R(0);
#pragma unroll
            for (int mm = 0; mm < P1; ++mm) sl += l_nbr[mm] * l_nbr[mm] / tw[mm];
            pfac = -R(0.5) * sl / detn;
          }
        }
        const R* tp = nullptr;
        const R* tpt = nullptr;
        if constexpr (TRC) tp = lin_traces<R>(md) + ((int64_t)nb * NF + (F ^ 1)) * (NCU * (1 + D)) * NFP + ff;
        if constexpr (TRT) tpt = dir_traces<R>(md) + ((int64_t)nb * NF + (F ^ 1)) * (NCU * (1 + D)) * NFP + ff;
#pragma unroll
        for (int c = 0; c < NCU; ++c) {
          const int64_t o = ((int64_t)nb * NCU + c) * NN + base;
          V sacc = T::mk(R(0));
          if constexpr (MODE == 2) {
            if constexpr (TRT) {
              sacc = T::mk(tp[c * NFP], tpt[c * NFP]);
            } else if constexpr (TRC) {
              R tv = R(0);
#pragma unroll
              for (int mm = 0; mm < P1; ++mm) tv += l_nbr[mm] * R(v[o + mm * SD]);
              sacc = T::mk(R(tp[c * NFP]), tv);
            } else {
#pragma unroll
              for (int mm = 0; mm < P1; ++mm) sacc += l_nbr[mm] * T::mk(R(u[o + mm * SD]), R(v[o + mm * SD]));
            }
          } else {
#pragma unroll
            for (int mm = 0; mm < P1; ++mm) sacc += l_nbr[mm] * R(u[o + mm * SD]);
          }
          up[c] = sacc;
#pragma unroll
          for (int k = 0; k < D; ++k) {
            V t = T::mk(R(0));
            if constexpr (HASQ) {
              const int64_t oq = (((int64_t)nb * NCU + c) * D + k) * NN + base;
              if constexpr (MODE == 2) {
                if constexpr (TRT) {
                  t = T::mk(tp[(NCU + c * D + k) * NFP], tpt[(NCU + c * D + k) * NFP]);
                } else if constexpr (TRC) {
                  R td = R(0);
                  if constexpr (PRB) {
                    td = pfac * T::tan(um[c]) * Nn[k];
                  } else {
#pragma unroll
                    for (int mm = 0; mm < P1; ++mm) td += l_nbr[mm] * dq[oq + mm * SD];
                  }
                  t = T::mk(R(tp[(NCU + c * D + k) * NFP]), td);
                } else {
#pragma unroll
                  for (int mm = 0; mm < P1; ++mm) t += l_nbr[mm] * T::mk(q[oq + mm * SD], dq[oq + mm * SD]);
                }
              } else {
#pragma unroll
                for (int mm = 0; mm < P1; ++mm) t += l_nbr[mm] * q[oq + mm * SD];
              }
            }
            qp[c][k] = t;
          }
        }
#pragma unroll
        for (int t = 0; t < NA; ++t) {
          R sacc = R(0);
          if (t < md.naux) {
            const double* ap = md.aux + ((int64_t)nb * md.naux + t) * NN + base;
#pragma unroll
            for (int mm = 0; mm < P1; ++mm) sacc += l_nbr[mm] * R(ap[mm * SD]);
          }
          ap2[t] = sacc;
        }
        if constexpr (KIND != K_USER) {
          half_normal_flux<KIND, D, V, R>(md.mu, md.naux, up, qp, ap2, n, Fh, true);
          penalty_flux<KIND, D, V, R>(md.mu, um, am, up, ap2, md.naux, n, Fh);
        } else {
          num_flux<KIND, D, V, R>(md.mu, md.naux, um, qm, am, up, qp, ap2, n, Fh);
        }
      } else {
        const int b = -(nb + 1);
        int tag = m.btag[b];
        tag = tag < 0 ? 0 : (tag >= md.nbc ? md.nbc - 1 : tag);
        const int kind = md.bc_kind[tag];
        if (kind == BC_DIRICHLET) {
          // the state outside is the data g (zero tangent); the linear operator (MODE 0) sees g = 0
          V ub[NCU];
#pragma unroll
          for (int c = 0; c < NCU; ++c)
            ub[c] = (MODE != 0 && md.bdata) ? T::mk(R(md.bdata[((int64_t)b * NCU + c) * NFP + ff])) : T::mk(R(0));
#ifdef LDG_USER_PHYSICS
          if constexpr (KIND == K_USER) boundary_state<KIND, D, V, R>(md.mu, md.naux, tag, um, qm, am, n, ub);
#endif
          num_flux<KIND, D, V, R>(md.mu, md.naux, um, qm, am, ub, qm, am, n, Fh);
        } else if (kind == BC_NEUMANN) {
#pragma unroll
          for (int c = 0; c < NCU; ++c)
            Fh[c] = (MODE == 1 && md.bdata) ? T::mk(R(md.bdata[((int64_t)b * NCU + c) * NFP + ff])) : T::mk(R(0));
        } else {
          V fl[NCU][D];
          phys_flux<KIND, D, V, R>(md.mu, md.naux, um, qm, am, fl);
#pragma unroll
          for (int c = 0; c < NCU; ++c) {
            V sacc = fl[c][0] * n[0];
#pragma unroll
            for (int k = 1; k < D; ++k) sacc += fl[c][k] * n[k];
            Fh[c] = sacc;
          }
        }
      }
      const R wds = wf * ds;
#pragma unroll
      for (int c = 0; c < NCU; ++c) {
        if constexpr (MODE == 2) s_Fh[e][F][c][ff] = wds * Fh[c].d;
        else s_Fh[e][F][c][ff] = wds * Fh[c];
      }
    }
  };
  auto faces = [&]() {
    for (int it = threadIdx.x; it < D * EPB * 2 * NFP; it += blockDim.x) {
      const int dir = it / (EPB * 2 * NFP), loc = it % (EPB * 2 * NFP);
      if (dir == 0) face_dir(std::integral_constant<int, 0>{}, loc);
      else if (dir == 1) face_dir(std::integral_constant<int, 1>{}, loc);
      else if constexpr (D == 3) face_dir(std::integral_constant<int, 2>{}, loc);
    }
  };
  // the tangent kernel visits the nodes first, so that the element's own q
  // lines, read again by its face points, are still in cache (64^3
  // Navier-Stokes FP64 tangent 9.9 -> 7.8 ms)
  constexpr bool VOLUME_FIRST = (MODE == 2);
  if constexpr (!VOLUME_FIRST) faces();

  // ---- volume: flux at the node, contravariant components to LDS, pointwise terms
  R r[NCU];
  int a[D];
  node_index<D, P1>(i, a);
  if (active) {
    R J[D][D], adj[D][D];
    geo_jac<D, P1, R, AFF>(s_g[el], s_c[el], a, J);
    const R det = adjugate<D, R>(J, adj);
    R wi = R(1);
#pragma unroll
    for (int k = 0; k < D; ++k) wi *= tw[a[k]];
    const R wdet = wi * det;

    V uu[NCU];
    V qq[NCU][D];
#pragma unroll
    for (int c = 0; c < NCU; ++c) {
      uu[c] = s_u[el][c][i];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        if constexpr (QLDS) {
          qq[c][k] = s_q[el][c * D + k][i];
        } else if constexpr (HASQ) {
          const int64_t o = ((K * NCU + c) * D + k) * NN + i;
          qq[c][k] = T::mk(q[o], dq[o]);
        } else {
          qq[c][k] = T::mk(R(0));
        }
      }
    }
    R aa[NA];
#pragma unroll
    for (int t = 0; t < NA; ++t) aa[t] = (t < md.naux) ? R(md.aux[(K * md.naux + t) * NN + i]) : R(0);
    V f[NCU][D];
    phys_flux<KIND, D, V, R>(md.mu, md.naux, uu, qq, aa, f);
    V sv[NCU];
    if constexpr (has_point_source<KIND, D>()) point_source<KIND, D, V, R>(md.mu, md.naux, uu, qq, aa, sv);
#pragma unroll
    for (int c = 0; c < NCU; ++c) {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        V sacc = adj[j][0] * f[c][0];
#pragma unroll
        for (int k = 1; k < D; ++k) sacc += adj[j][k] * f[c][k];
        if constexpr (MODE == 2) s_F[el][c][j][i] = wi * sacc.d;
        else if constexpr (EXT) Fout[((K * NCU + c) * D + j) * NN + i] = float(wi * sacc);   // divergence done outside
        else s_F[el][c][j][i] = wi * sacc;
      }
      R rc;
      if constexpr (MODE == 2) {
        rc = R(tm.a0) * wdet * uu[c].d;
      } else {
        const int64_t o = (K * NCU + c) * NN + i;
        R t = R(tm.a0) * uu[c];
        if (tm.r1) t -= R(tm.c1) * R(tm.r1[o]);
        if (tm.r2) t -= R(tm.c2) * R(tm.r2[o]);
        rc = wdet * t;
        if constexpr (KIND == K_POISSON) rc += wdet * R(md.mu[2]) * uu[c];
        if constexpr (MODE == 1) {
          if (md.src) rc -= wdet * R(md.src[o]);
        }
      }
      if constexpr (has_point_source<KIND, D>()) {
        if constexpr (MODE == 2) rc -= wdet * sv[c].d;
        else rc -= wdet * sv[c];
      }
      r[c] = rc;
    }
  }
  if constexpr (VOLUME_FIRST) faces();
  __syncthreads();
  if (!active) return;

  // ---- contraction with the transposed derivative matrix, lifting, store
#pragma unroll
  for (int c = 0; c < NCU; ++c) {
    R acc = r[c];
#pragma unroll
    for (int j = 0; j < D && !EXT; ++j) {
      const int sj = stride_c(P1, j);
      const int b0 = i - a[j] * sj;
      R sacc = R(0);
#pragma unroll
      for (int mm = 0; mm < P1; ++mm) sacc += tD[mm * P1 + a[j]] * s_F[el][c][j][b0 + mm * sj];
      acc -= sacc;
    }
#pragma unroll
    for (int F = 0; F < NF; ++F) {
      const int dir = F >> 1, side = F & 1;
      acc += tl[side * P1 + a[dir]] * s_Fh[el][F][c][face_index_of_node<D, P1>(a, dir)];
    }
    const int64_t o = (K * NCU + c) * NN + i;
    double res = double(acc);
    if (dterm) res += dterm[o];
    out[o] = res;
  }
}

}  // namespace ldg
