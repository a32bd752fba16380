// LDG operator kernels for gfx950: the local gradient q (Eq. 1a in weak form),
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
// live in LDS.  Work-groups are mapped to elements so that each of the eight
// XCDs (which receive work-groups round-robin) walks a contiguous range of
// elements and finds most neighbours in its own L2.
#include <type_traits>

#include "ldg_physics.hpp"

namespace ldg {

template <class R> struct TabOf;
template <> struct TabOf<double> { using T = BasisTab; };
template <> struct TabOf<float> { using T = BasisTabF; };

// Elements per work-group: fill 256 threads, bounded by an LDS budget per group.
template <int NN, int BYTES_PER_ELEM>
constexpr int pick_epb() {
  int e = 256 / NN;
  if (e < 1) e = 1;
  while (e > 1 && e * BYTES_PER_ELEM > 40 * 1024) --e;
  return e;
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

// work-group -> element block, XCD-aware (work-group b runs on XCD b % 8)
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
template <int D, int J, class R>
__device__ inline void jac_col(const double* __restrict__ c, const R* xi, R* col) {
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
template <int D, int DIR, class R>
__device__ inline void face_normal(const double* __restrict__ c, const R* xi, int side, R* N) {
  const R s = side ? R(1) : R(-1);
  if constexpr (D == 2) {
    constexpr int T = 1 - DIR;
    R col[2];
    jac_col<2, T, R>(c, xi, col);
    if constexpr (DIR == 0) { N[0] = s * col[1]; N[1] = -s * col[0]; }
    else { N[0] = -s * col[1]; N[1] = s * col[0]; }
  } else {
    // row DIR of adj = col(DIR+1) x col(DIR+2) (cyclic)
    constexpr int A = (DIR + 1) % 3, B = (DIR + 2) % 3;
    R a[3], b[3];
    jac_col<3, A, R>(c, xi, a);
    jac_col<3, B, R>(c, xi, b);
    N[0] = s * (a[1] * b[2] - a[2] * b[1]);
    N[1] = s * (a[2] * b[0] - a[0] * b[2]);
    N[2] = s * (a[0] * b[1] - a[1] * b[0]);
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

template <int KIND, int D, int P1, class R>
struct GradCfg {
  static constexpr int NCU = Phys<KIND, D>::NCU, NN = ipow(P1, D), NFP = ipow(P1, D - 1), NF = 2 * D, NV = 1 << D;
  static constexpr int BYTES = sizeof(R) * (NCU * NN + NF * NCU * D * NFP) + 8 * NV * D;
  static constexpr int EPB = pick_epb<NN, BYTES>();
};

template <int KIND, int D, int P1, class R, int MODE>
struct ResidCfg {
  using PH = Phys<KIND, D>;
  using V = typename std::conditional<MODE == 2, Dl<R>, R>::type;
  static constexpr int NCU = PH::NCU, NN = ipow(P1, D), NFP = ipow(P1, D - 1), NF = 2 * D, NV = 1 << D;
  static constexpr bool HASQ = PH::HASQ;
  static constexpr int NQ = HASQ ? NCU * D : 1;
  static constexpr int BYTES = sizeof(V) * (NCU * NN + (HASQ ? NCU * D * NN : 0)) +
                               sizeof(R) * (NCU * D * NN + NF * NCU * NFP) + 8 * NV * D;
  static constexpr int EPB = pick_epb<NN, BYTES>();
};

// ============================================================================
// Local gradient: q = M^-1 [ (u, div r) - <uhat n, r> ], evaluated in the
// equivalent strong form q = -grad u + M^-1 <(u- - uhat) n, r> (integration by
// parts is exact under the collocated Gauss rule for multilinear elements).
// DATA = true: Dirichlet uhat = g from bdata (nonlinear models); false:
// homogeneous (tangents, and linear models whose data enter through qoff).
// ============================================================================
template <int KIND, int D, int P1, class R, bool DATA, bool EXT = false>
__global__ void __launch_bounds__(256)
k_grad(MeshDev m, typename TabOf<R>::T tab, ModelDev md, const double* __restrict__ u, R* __restrict__ q,
       const double* __restrict__ qoff, const float* __restrict__ dux = nullptr) {
  using C = GradCfg<KIND, D, P1, R>;
  constexpr int NCU = C::NCU, NN = C::NN, NFP = C::NFP, NF = C::NF, NV = C::NV, EPB = C::EPB;
  using L = TabLayout<P1>;
  __shared__ R s_tab[L::SIZE];
  __shared__ R s_u[EPB][NCU][NN];
  __shared__ R s_L[EPB][NF][NCU][D][NFP];
  __shared__ double s_c[EPB][NV * D];

  const int64_t eb = xcd_block(blockIdx.x, gridDim.x);
  const int el = threadIdx.x / NN, i = threadIdx.x % NN;
  const int64_t K = eb * EPB + el;
  const bool active = K < m.E;
  stage_tables<P1, R>(tab, s_tab);
  if (active) {
#pragma unroll
    for (int c = 0; c < NCU; ++c) s_u[el][c][i] = R(u[(K * NCU + c) * NN + i]);
    for (int t = i; t < NV * D; t += NN) s_c[el][t] = m.coef[K * NV * D + t];
  }
  __syncthreads();
  const R* tx = s_tab + L::X;
  const R* tw = s_tab + L::W;
  const R* tD = s_tab + L::DM;
  const R* tl = s_tab + L::LF;

  // ---- faces, one reference direction at a time
  auto face_dir = [&](auto dirc) {
    constexpr int DIR = decltype(dirc)::value;
    constexpr int T0 = Tang<D, DIR>::T0, T1 = Tang<D, DIR>::T1;
    constexpr int SD = stride_c(P1, DIR);
    for (int it = threadIdx.x; it < EPB * 2 * NFP; it += blockDim.x) {
      const int e = it / (2 * NFP), side = (it / NFP) & 1, f = it % NFP;
      const int64_t Ke = eb * EPB + e;
      if (Ke >= m.E) continue;
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
          const double* un = u + ((int64_t)nb * NCU + c) * NN + base;
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
          if (kind == LDG_BC_DIRICHLET)
            uh[c] = (DATA && md.bdata) ? R(md.bdata[((int64_t)b * NCU + c) * NFP + f]) : R(0);
          else
            uh[c] = um[c];
        }
      }
      R xi[D];
      xi[DIR] = side ? R(1) : R(-1);
      xi[T0] = tx[t0];
      if constexpr (D == 3) xi[T1] = tx[t1];
      R N[D];
      face_normal<D, DIR, R>(s_c[e], xi, side, N);
#pragma unroll
      for (int c = 0; c < NCU; ++c)
#pragma unroll
        for (int k = 0; k < D; ++k) s_L[e][F][c][k][f] = (um[c] - uh[c]) * N[k];
    }
  };
  face_dir(std::integral_constant<int, 0>{});
  face_dir(std::integral_constant<int, 1>{});
  if constexpr (D == 3) face_dir(std::integral_constant<int, 2>{});
  __syncthreads();
  if (!active) return;

  int a[D];
  node_index<D, P1>(i, a);
  R xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = tx[a[k]];
  R J[D][D], adj[D][D];
  jacobian_at<D, R>(s_c[el], xi, J);
  const R det = adjugate<D, R>(J, adj);
  const R idet = R(1) / det;
  R liftw[NF];      // l_{a_dir}(side) / (w_{a_dir} det)
  int fidx[D];
#pragma unroll
  for (int F = 0; F < NF; ++F) liftw[F] = tl[(F & 1) * P1 + a[F >> 1]] / tw[a[F >> 1]] * idet;
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
template <int KIND, int D, int P1, class R, int MODE, bool EXT = false>
__global__ void __launch_bounds__(256)
k_resid(MeshDev m, typename TabOf<R>::T tab, ModelDev md, TimeDev tm, const double* __restrict__ u,
        const R* __restrict__ q, const double* __restrict__ v, const R* __restrict__ dq,
        const double* __restrict__ dterm, double* __restrict__ out, float* __restrict__ Fout = nullptr) {
  using C = ResidCfg<KIND, D, P1, R, MODE>;
  using V = typename C::V;
  using T = VT<V>;
  constexpr int NCU = C::NCU, NN = C::NN, NFP = C::NFP, NF = C::NF, NV = C::NV, EPB = C::EPB, NQ = C::NQ;
  constexpr bool HASQ = C::HASQ;
  constexpr int NA = Phys<KIND, D>::NAUX > 0 ? Phys<KIND, D>::NAUX : 1;
  using L = TabLayout<P1>;
  __shared__ R s_tab[L::SIZE];
  __shared__ V s_u[EPB][NCU][NN];
  __shared__ V s_q[EPB][NQ][HASQ ? NN : 1];
  __shared__ R s_F[EPB][NCU][D][NN];
  __shared__ R s_Fh[EPB][NF][NCU][NFP];
  __shared__ double s_c[EPB][NV * D];

  const int64_t eb = xcd_block(blockIdx.x, gridDim.x);
  const int el = threadIdx.x / NN, i = threadIdx.x % NN;
  const int64_t K = eb * EPB + el;
  const bool active = K < m.E;
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
    if constexpr (HASQ) {
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const int64_t o = (K * NQ + c) * NN + i;
        if constexpr (MODE == 2) s_q[el][c][i] = T::mk(q[o], dq[o]);
        else s_q[el][c][i] = q[o];
      }
    }
    for (int t = i; t < NV * D; t += NN) s_c[el][t] = m.coef[K * NV * D + t];
  }
  __syncthreads();
  const R* tx = s_tab + L::X;
  const R* tw = s_tab + L::W;
  const R* tD = s_tab + L::DM;
  const R* tl = s_tab + L::LF;

  // ---- faces: numerical flux times w ds, to LDS, one reference direction at a time
  auto face_dir = [&](auto dirc) {
    constexpr int DIR = decltype(dirc)::value;
    constexpr int T0 = Tang<D, DIR>::T0, T1 = Tang<D, DIR>::T1;
    constexpr int SD = stride_c(P1, DIR);
    for (int it = threadIdx.x; it < EPB * 2 * NFP; it += blockDim.x) {
      const int e = it / (2 * NFP), side = (it / NFP) & 1, ff = it % NFP;
      const int64_t Ke = eb * EPB + e;
      if (Ke >= m.E) continue;
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
          if constexpr (HASQ) {
#pragma unroll
            for (int mm = 0; mm < P1; ++mm) t += l_own[mm] * s_q[e][c * D + k][base + mm * SD];
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
      R xi2[D];
      xi2[DIR] = side ? R(1) : R(-1);
      xi2[T0] = tx[t0];
      if constexpr (D == 3) xi2[T1] = tx[t1];
      R N[D], n[D];
      face_normal<D, DIR, R>(s_c[e], xi2, side, N);
      R ds = R(0);
#pragma unroll
      for (int k = 0; k < D; ++k) ds += N[k] * N[k];
      ds = vsqrt(ds);
      const R ids = R(1) / ds;
#pragma unroll
      for (int k = 0; k < D; ++k) n[k] = N[k] * ids;
      R wf = tw[t0];
      if constexpr (D == 3) wf *= tw[t1];

      const int F = 2 * DIR + side;
      V Fh[NCU];
      const int nb = m.nbr[Ke * NF + F];
      if (nb >= 0) {
        V up[NCU], qp[NCU][D];
        R ap2[NA];
#pragma unroll
        for (int c = 0; c < NCU; ++c) {
          const int64_t o = ((int64_t)nb * NCU + c) * NN + base;
          V sacc = T::mk(R(0));
#pragma unroll
          for (int mm = 0; mm < P1; ++mm) {
            if constexpr (MODE == 2) sacc += l_nbr[mm] * T::mk(R(u[o + mm * SD]), R(v[o + mm * SD]));
            else sacc += l_nbr[mm] * R(u[o + mm * SD]);
          }
          up[c] = sacc;
#pragma unroll
          for (int k = 0; k < D; ++k) {
            V t = T::mk(R(0));
            if constexpr (HASQ) {
              const int64_t oq = (((int64_t)nb * NCU + c) * D + k) * NN + base;
#pragma unroll
              for (int mm = 0; mm < P1; ++mm) {
                if constexpr (MODE == 2) t += l_nbr[mm] * T::mk(q[oq + mm * SD], dq[oq + mm * SD]);
                else t += l_nbr[mm] * q[oq + mm * SD];
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
        num_flux<KIND, D, V, R>(md.mu, md.naux, um, qm, am, up, qp, ap2, n, Fh);
      } else {
        const int b = -(nb + 1);
        int tag = m.btag[b];
        tag = tag < 0 ? 0 : (tag >= md.nbc ? md.nbc - 1 : tag);
        const int kind = md.bc_kind[tag];
        if (kind == LDG_BC_DIRICHLET) {
          // the state outside is the data g (zero tangent); the linear operator (MODE 0) sees g = 0
          V ub[NCU];
#pragma unroll
          for (int c = 0; c < NCU; ++c)
            ub[c] = (MODE != 0 && md.bdata) ? T::mk(R(md.bdata[((int64_t)b * NCU + c) * NFP + ff])) : T::mk(R(0));
          num_flux<KIND, D, V, R>(md.mu, md.naux, um, qm, am, ub, qm, am, n, Fh);
        } else if (kind == LDG_BC_NEUMANN) {
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
  face_dir(std::integral_constant<int, 0>{});
  face_dir(std::integral_constant<int, 1>{});
  if constexpr (D == 3) face_dir(std::integral_constant<int, 2>{});

  // ---- volume: flux at the node, contravariant components to LDS, pointwise terms
  R r[NCU];
  int a[D];
  node_index<D, P1>(i, a);
  if (active) {
    R xi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xi[k] = tx[a[k]];
    R J[D][D], adj[D][D];
    jacobian_at<D, R>(s_c[el], xi, J);
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
        if constexpr (HASQ) qq[c][k] = s_q[el][c * D + k][i];
        else qq[c][k] = T::mk(R(0));
      }
    }
    R aa[NA];
#pragma unroll
    for (int t = 0; t < NA; ++t) aa[t] = (t < md.naux) ? R(md.aux[(K * md.naux + t) * NN + i]) : R(0);
    V f[NCU][D];
    phys_flux<KIND, D, V, R>(md.mu, md.naux, uu, qq, aa, f);
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
      r[c] = rc;
    }
  }
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

// ============================================================================
// host dispatch
// ============================================================================
template <int KIND, int D, int P1, class R>
static ldg_status launch_grad(const Model& md, const double* u, void* q, bool with_data, hipStream_t s) {
  // linear models: homogeneous kernel + boundary-data offset; nonlinear: data in the kernel
  const bool in_kernel_data = with_data && !Phys<KIND, D>::LINEAR;
  const double* qoff = (with_data && Phys<KIND, D>::LINEAR) ? md.d_qg : nullptr;
  constexpr int NN = GradCfg<KIND, D, P1, R>::NN, EPB = GradCfg<KIND, D, P1, R>::EPB;
  const Mesh& m = *md.mesh;
  const int nblk = (int)((m.E + EPB - 1) / EPB);
  typename TabOf<R>::T tab;
  if constexpr (std::is_same<R, double>::value) tab = m.tab; else tab = m.tabf;
  if (in_kernel_data)
    hipLaunchKernelGGL((k_grad<KIND, D, P1, R, true>), dim3(nblk), dim3(EPB * NN), 0, s, m.dev(), tab, md.dev(), u,
                       (R*)q, qoff);
  else
    hipLaunchKernelGGL((k_grad<KIND, D, P1, R, false>), dim3(nblk), dim3(EPB * NN), 0, s, m.dev(), tab, md.dev(), u,
                       (R*)q, qoff);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

template <int KIND, int D, int P1, class R, int MODE>
static ldg_status launch_resid(const Model& md, const TimeDev& t, const double* u, const void* q, const double* v,
                               const void* dq, const double* dterm, double* out, hipStream_t s) {
  constexpr int NN = ResidCfg<KIND, D, P1, R, MODE>::NN, EPB = ResidCfg<KIND, D, P1, R, MODE>::EPB;
  const Mesh& m = *md.mesh;
  const int nblk = (int)((m.E + EPB - 1) / EPB);
  typename TabOf<R>::T tab;
  if constexpr (std::is_same<R, double>::value) tab = m.tab; else tab = m.tabf;
  hipLaunchKernelGGL((k_resid<KIND, D, P1, R, MODE>), dim3(nblk), dim3(EPB * NN), 0, s, m.dev(), tab, md.dev(), t, u,
                     (const R*)q, v, (const R*)dq, dterm, out);
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

// compile-time dispatch over (kind, nd, p+1)
template <template <int, int, int> class F, class... Args>
static ldg_status dispatch(int kind, int nd, int p1, Args&&... args) {
#define LDG_CASE(KI, DD, PP) \
  if (kind == KI && nd == DD && p1 == PP) return F<KI, DD, PP>::run(args...);
#define LDG_CASES_K(KI)                                                                        \
  LDG_CASE(KI, 2, 2) LDG_CASE(KI, 2, 3) LDG_CASE(KI, 2, 4) LDG_CASE(KI, 2, 5) LDG_CASE(KI, 3, 2) \
  LDG_CASE(KI, 3, 3) LDG_CASE(KI, 3, 4)
  LDG_CASES_K(0)
  LDG_CASES_K(1)
  LDG_CASES_K(2)
  LDG_CASES_K(3)
#undef LDG_CASES_K
#undef LDG_CASE
  set_error("no compiled kernel for this (model, nd, p)");
  return LDG_EUNSUPPORTED;
}

template <int KI, int DD, int PP>
struct GradOp {
  static ldg_status run(const Model& md, const double* u, void* q, bool fp32, bool with_data, hipStream_t s) {
    if constexpr (KI == K_EULER) {
      return LDG_OK;
    } else {
      if (fp32) return launch_grad<KI, DD, PP, float>(md, u, q, with_data, s);
      return launch_grad<KI, DD, PP, double>(md, u, q, with_data, s);
    }
  }
};

template <int KI, int DD, int PP>
struct ResidOp {
  static ldg_status run(const Model& md, const TimeDev& t, const double* u, const void* q, double* out, bool fp32,
                        bool with_data, hipStream_t s) {
    if constexpr (KI <= K_CONVDIFF) {
      const double* dt = with_data ? md.d_dterm : nullptr;
      if (fp32) return launch_resid<KI, DD, PP, float, 0>(md, t, u, q, nullptr, nullptr, dt, out, s);
      return launch_resid<KI, DD, PP, double, 0>(md, t, u, q, nullptr, nullptr, dt, out, s);
    } else {
      if (fp32) return launch_resid<KI, DD, PP, float, 1>(md, t, u, q, nullptr, nullptr, nullptr, out, s);
      return launch_resid<KI, DD, PP, double, 1>(md, t, u, q, nullptr, nullptr, nullptr, out, s);
    }
  }
};

template <int KI, int DD, int PP>
struct TangentOp {
  static ldg_status run(const Model& md, const TimeDev& t, const double* u, const void* q, const double* v,
                        const void* dq, double* out, bool fp32, hipStream_t s) {
    if constexpr (KI <= K_CONVDIFF) {
      set_error("tangent kernel requested for a linear model");
      return LDG_EINVAL;
    } else {
      if (fp32) return launch_resid<KI, DD, PP, float, 2>(md, t, u, q, v, dq, nullptr, out, s);
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

ldg_status op_grad_ext(const Model& md, const double* u, const float* du, float* q, hipStream_t s) {
  return dispatch<GradExtOp>(md.kind, md.mesh->nd, md.mesh->p1, md, u, du, q, s);
}
ldg_status op_resid_ext(const Model& md, const TimeDev& t, const double* u, const float* q, float* F, double* out,
                        hipStream_t s) {
  return dispatch<ResidExtOp>(md.kind, md.mesh->nd, md.mesh->p1, md, t, u, q, F, out, s);
}

ldg_status op_grad(const Model& md, const double* u, void* q, bool fp32, bool with_data, hipStream_t s) {
  return dispatch<GradOp>(md.kind, md.mesh->nd, md.mesh->p1, md, u, q, fp32, with_data, s);
}

ldg_status op_resid(const Model& md, const TimeDev& t, const double* u, const void* q, double* out, bool fp32,
                    bool with_data, hipStream_t s) {
  return dispatch<ResidOp>(md.kind, md.mesh->nd, md.mesh->p1, md, t, u, q, out, fp32, with_data, s);
}

ldg_status op_jvp_nonlinear(const Model& md, const TimeDev& t, const double* u, const void* q, const double* v,
                            const void* dq, double* out, bool fp32, hipStream_t s) {
  return dispatch<TangentOp>(md.kind, md.mesh->nd, md.mesh->p1, md, t, u, q, v, dq, out, fp32, s);
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
