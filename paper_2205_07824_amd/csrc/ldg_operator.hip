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

// node multi-index of flat node i (first direction fastest)
template <int D, int P1>
__device__ inline void node_index(int i, int* a) {
#pragma unroll
  for (int k = 0; k < D; ++k) { a[k] = i % P1; i /= P1; }
}

// tangential indices of face point f on a face normal to dir; returns the
// flat node offset of the face point's line (the dir index set to 0)
template <int D, int P1>
__device__ inline int face_line(int dir, int f, int* tix) {
  int off = 0, t = 0, ff = f;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    if (k == dir) continue;
    tix[t] = ff % P1;
    ff /= P1;
    off += tix[t] * ipow(P1, k);
    ++t;
  }
  return off;
}

// tangential flat index of node a[] with respect to direction dir
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

__device__ inline int stride_of(int P1, int k) { return k == 0 ? 1 : (k == 1 ? P1 : P1 * P1); }

// ============================================================================
// Local gradient: q = M^-1 [ (u, div r) - <uhat n, r> ], evaluated in the
// equivalent strong form q = -grad u + M^-1 <(u- - uhat) n, r> (integration by
// parts is exact under the collocated Gauss rule for multilinear elements).
// DATA = true: Dirichlet uhat = g from bdata (nonlinear models); false:
// homogeneous (tangents, and linear models whose data enter through qoff).
// ============================================================================
template <int KIND, int D, int P1, class R, bool DATA>
__global__ void __launch_bounds__(256)
k_grad(MeshDev m, typename TabOf<R>::T tab, ModelDev md, const double* __restrict__ u, R* __restrict__ q,
       const double* __restrict__ qoff) {
  using PH = Phys<KIND, D>;
  constexpr int NCU = PH::NCU, NN = ipow(P1, D), NFP = ipow(P1, D - 1), NF = 2 * D, NV = 1 << D;
  constexpr int BYTES = sizeof(R) * (NCU * NN + NF * NCU * D * NFP) + 8 * NV * D;
  constexpr int EPB = pick_epb<NN, BYTES>();
  __shared__ R s_u[EPB][NCU][NN];
  __shared__ R s_L[EPB][NF][NCU][D][NFP];
  __shared__ double s_c[EPB][NV * D];

  const int el = threadIdx.x / NN, i = threadIdx.x % NN;
  const int64_t K = (int64_t)blockIdx.x * EPB + el;
  const bool active = K < m.E;
  if (active) {
#pragma unroll
    for (int c = 0; c < NCU; ++c) s_u[el][c][i] = R(u[(K * NCU + c) * NN + i]);
    for (int t = i; t < NV * D; t += NN) s_c[el][t] = m.coef[K * NV * D + t];
  }
  __syncthreads();

  if (active) {
    for (int fp = i; fp < NF * NFP; fp += NN) {
      const int F = fp / NFP, f = fp % NFP, dir = F >> 1, side = F & 1;
      int tix[2] = {0, 0};
      const int base = face_line<D, P1>(dir, f, tix);
      const int sd = stride_of(P1, dir);
      R um[NCU], uh[NCU];
#pragma unroll
      for (int c = 0; c < NCU; ++c) {
        R s = R(0);
#pragma unroll
        for (int mm = 0; mm < P1; ++mm) s += tab.lf[side][mm] * s_u[el][c][base + mm * sd];
        um[c] = s;
      }
      const int nb = m.nbr[K * NF + F];
      if (nb >= 0) {
#pragma unroll
        for (int c = 0; c < NCU; ++c) {
          R s = R(0);
          const double* un = u + ((int64_t)nb * NCU + c) * NN + base;
#pragma unroll
          for (int mm = 0; mm < P1; ++mm) s += tab.lf[1 - side][mm] * R(un[mm * sd]);
          uh[c] = R(0.5) * (um[c] + s);
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
#pragma unroll
      for (int k = 0, t = 0; k < D; ++k) xi[k] = (k == dir) ? (side ? R(1) : R(-1)) : tab.x[tix[t++]];
      R J[D][D], N[D];
      jacobian_at<D, R>(s_c[el], xi, J);
      scaled_normal<D, R>(J, dir, side, N);
#pragma unroll
      for (int c = 0; c < NCU; ++c)
#pragma unroll
        for (int k = 0; k < D; ++k) s_L[el][F][c][k][f] = (um[c] - uh[c]) * N[k];
    }
  }
  __syncthreads();
  if (!active) return;

  int a[D];
  node_index<D, P1>(i, a);
  R xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = tab.x[a[k]];
  R J[D][D], adj[D][D];
  jacobian_at<D, R>(s_c[el], xi, J);
  const R det = adjugate<D, R>(J, adj);
  const R idet = R(1) / det;
#pragma unroll
  for (int c = 0; c < NCU; ++c) {
    R du[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int sj = stride_of(P1, j);
      const int b0 = i - a[j] * sj;
      R s = R(0);
#pragma unroll
      for (int mm = 0; mm < P1; ++mm) s += tab.D[a[j]][mm] * s_u[el][c][b0 + mm * sj];
      du[j] = s;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
      R g = R(0);
#pragma unroll
      for (int j = 0; j < D; ++j) g += adj[j][k] * du[j];
      R qv = -g * idet;
#pragma unroll
      for (int F = 0; F < NF; ++F) {
        const int dir = F >> 1, side = F & 1;
        qv += tab.lf[side][a[dir]] / (tab.w[a[dir]] * det) * s_L[el][F][c][k][face_index_of_node<D, P1>(a, dir)];
      }
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
template <int KIND, int D, int P1, class R, int MODE>
__global__ void __launch_bounds__(256)
k_resid(MeshDev m, typename TabOf<R>::T tab, ModelDev md, TimeDev tm, const double* __restrict__ u,
        const R* __restrict__ q, const double* __restrict__ v, const R* __restrict__ dq,
        const double* __restrict__ dterm, double* __restrict__ out) {
  using PH = Phys<KIND, D>;
  using V = typename std::conditional<MODE == 2, Dl<R>, R>::type;
  using T = VT<V>;
  constexpr int NCU = PH::NCU, NN = ipow(P1, D), NFP = ipow(P1, D - 1), NF = 2 * D, NV = 1 << D;
  constexpr bool HASQ = PH::HASQ;
  constexpr int NQ = HASQ ? NCU * D : 1;
  constexpr int NA = PH::NAUX > 0 ? PH::NAUX : 1;
  constexpr int BYTES = sizeof(V) * (NCU * NN + (HASQ ? NCU * D * NN : 0)) +
                        sizeof(R) * (NCU * D * NN + NF * NCU * NFP) + 8 * NV * D;
  constexpr int EPB = pick_epb<NN, BYTES>();
  __shared__ V s_u[EPB][NCU][NN];
  __shared__ V s_q[EPB][NQ][HASQ ? NN : 1];
  __shared__ R s_F[EPB][NCU][D][NN];
  __shared__ R s_Fh[EPB][NF][NCU][NFP];
  __shared__ double s_c[EPB][NV * D];

  const int el = threadIdx.x / NN, i = threadIdx.x % NN;
  const int64_t K = (int64_t)blockIdx.x * EPB + el;
  const bool active = K < m.E;

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

  R r[NCU];
  int a[D];
  node_index<D, P1>(i, a);
  if (active) {
    // ---- volume: flux at the node, contravariant components to LDS
    R xi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xi[k] = tab.x[a[k]];
    R J[D][D], adj[D][D];
    jacobian_at<D, R>(s_c[el], xi, J);
    const R det = adjugate<D, R>(J, adj);
    R wi = R(1);
#pragma unroll
    for (int k = 0; k < D; ++k) wi *= tab.w[a[k]];
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
        V s = adj[j][0] * f[c][0];
#pragma unroll
        for (int k = 1; k < D; ++k) s += adj[j][k] * f[c][k];
        if constexpr (MODE == 2) s_F[el][c][j][i] = wi * s.d;
        else s_F[el][c][j][i] = wi * s;
      }
      // pointwise terms: time wrapper, source
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

    // ---- faces: numerical flux times w ds, to LDS
    for (int fp = i; fp < NF * NFP; fp += NN) {
      const int F = fp / NFP, ff = fp % NFP, dir = F >> 1, side = F & 1;
      int tix[2] = {0, 0};
      const int base = face_line<D, P1>(dir, ff, tix);
      const int sd = stride_of(P1, dir);
      V um[NCU], qm[NCU][D];
      R am[NA];
#pragma unroll
      for (int c = 0; c < NCU; ++c) {
        V s = T::mk(R(0));
#pragma unroll
        for (int mm = 0; mm < P1; ++mm) s += tab.lf[side][mm] * s_u[el][c][base + mm * sd];
        um[c] = s;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          V t = T::mk(R(0));
          if constexpr (HASQ) {
#pragma unroll
            for (int mm = 0; mm < P1; ++mm) t += tab.lf[side][mm] * s_q[el][c * D + k][base + mm * sd];
          }
          qm[c][k] = t;
        }
      }
#pragma unroll
      for (int t = 0; t < NA; ++t) {
        R s = R(0);
        if (t < md.naux) {
          const double* ap = md.aux + (K * md.naux + t) * NN + base;
#pragma unroll
          for (int mm = 0; mm < P1; ++mm) s += tab.lf[side][mm] * R(ap[mm * sd]);
        }
        am[t] = s;
      }
      R xi2[D];
#pragma unroll
      for (int k = 0, t = 0; k < D; ++k) xi2[k] = (k == dir) ? (side ? R(1) : R(-1)) : tab.x[tix[t++]];
      R J2[D][D], N[D], n[D];
      jacobian_at<D, R>(s_c[el], xi2, J2);
      scaled_normal<D, R>(J2, dir, side, N);
      R ds = R(0);
#pragma unroll
      for (int k = 0; k < D; ++k) ds += N[k] * N[k];
      ds = vsqrt(ds);
#pragma unroll
      for (int k = 0; k < D; ++k) n[k] = N[k] / ds;
      R wf = R(1);
#pragma unroll
      for (int t = 0; t < D - 1; ++t) wf *= tab.w[tix[t]];

      V Fh[NCU];
      const int nb = m.nbr[K * NF + F];
      if (nb >= 0) {
        V up[NCU], qp[NCU][D];
        R ap2[NA];
        const int os = 1 - side;
#pragma unroll
        for (int c = 0; c < NCU; ++c) {
          const int64_t o = ((int64_t)nb * NCU + c) * NN + base;
          V s = T::mk(R(0));
#pragma unroll
          for (int mm = 0; mm < P1; ++mm) {
            if constexpr (MODE == 2) s += tab.lf[os][mm] * T::mk(R(u[o + mm * sd]), R(v[o + mm * sd]));
            else s += tab.lf[os][mm] * R(u[o + mm * sd]);
          }
          up[c] = s;
#pragma unroll
          for (int k = 0; k < D; ++k) {
            V t = T::mk(R(0));
            if constexpr (HASQ) {
              const int64_t oq = (((int64_t)nb * NCU + c) * D + k) * NN + base;
#pragma unroll
              for (int mm = 0; mm < P1; ++mm) {
                if constexpr (MODE == 2) t += tab.lf[os][mm] * T::mk(q[oq + mm * sd], dq[oq + mm * sd]);
                else t += tab.lf[os][mm] * q[oq + mm * sd];
              }
            }
            qp[c][k] = t;
          }
        }
#pragma unroll
        for (int t = 0; t < NA; ++t) {
          R s = R(0);
          if (t < md.naux) {
            const double* ap = md.aux + ((int64_t)nb * md.naux + t) * NN + base;
#pragma unroll
            for (int mm = 0; mm < P1; ++mm) s += tab.lf[os][mm] * R(ap[mm * sd]);
          }
          ap2[t] = s;
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
            V s = fl[c][0] * n[0];
#pragma unroll
            for (int k = 1; k < D; ++k) s += fl[c][k] * n[k];
            Fh[c] = s;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < NCU; ++c) {
        if constexpr (MODE == 2) s_Fh[el][F][c][ff] = wf * ds * Fh[c].d;
        else s_Fh[el][F][c][ff] = wf * ds * Fh[c];
      }
    }
  }
  __syncthreads();
  if (!active) return;

  // ---- contraction with the transposed derivative matrix, lifting, store
#pragma unroll
  for (int c = 0; c < NCU; ++c) {
    R acc = r[c];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int sj = stride_of(P1, j);
      const int b0 = i - a[j] * sj;
      R s = R(0);
#pragma unroll
      for (int mm = 0; mm < P1; ++mm) s += tab.D[mm][a[j]] * s_F[el][c][j][b0 + mm * sj];
      acc -= s;
    }
#pragma unroll
    for (int F = 0; F < NF; ++F) {
      const int dir = F >> 1, side = F & 1;
      acc += tab.lf[side][a[dir]] * s_Fh[el][F][c][face_index_of_node<D, P1>(a, dir)];
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
  constexpr int NN = ipow(P1, D), NCU = Phys<KIND, D>::NCU, NFP = ipow(P1, D - 1), NF = 2 * D, NV = 1 << D;
  constexpr int BYTES = sizeof(R) * (NCU * NN + NF * NCU * D * NFP) + 8 * NV * D;
  constexpr int EPB = pick_epb<NN, BYTES>();
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
  using PH = Phys<KIND, D>;
  using V = typename std::conditional<MODE == 2, Dl<R>, R>::type;
  constexpr int NN = ipow(P1, D), NCU = PH::NCU, NFP = ipow(P1, D - 1), NF = 2 * D, NV = 1 << D;
  constexpr bool HASQ = PH::HASQ;
  constexpr int BYTES = sizeof(V) * (NCU * NN + (HASQ ? NCU * D * NN : 0)) +
                        sizeof(R) * (NCU * D * NN + NF * NCU * NFP) + 8 * NV * D;
  constexpr int EPB = pick_epb<NN, BYTES>();
  const Mesh& m = *md.mesh;
  const int nblk = (int)((m.E + EPB - 1) / EPB);
  typename TabOf<R>::T tab;
  if constexpr (std::is_same<R, double>::value) tab = m.tab; else tab = m.tabf;
  hipLaunchKernelGGL((k_resid<KIND, D, P1, R, MODE>), dim3(nblk), dim3(EPB * NN), 0, s, m.dev(), tab, md.dev(), t, u,
                     (const R*)q, v, (const R*)dq, dterm, out);
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
