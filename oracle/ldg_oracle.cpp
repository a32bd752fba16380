// Plain, slow FP64 CPU oracle of the local discontinuous Galerkin (LDG)
// operator of the parametrized first-order PDE system (Section 2.1, Eq. 1a-1b)
// and of its Jacobian.  TEST INFRASTRUCTURE ONLY: nothing in the product path
// links or calls this file; it exists so that the HIP library can be checked
// against an independent, obviously correct implementation.
//
// Everything here follows the plain definitions, without blocking, fusion or
// sum factorization:
//   * Gauss-Legendre points by Newton iteration on the Legendre recurrence;
//   * Lagrange basis on the (p+1) Gauss-Legendre nodes by the product formula;
//   * multilinear element maps, explicit Jacobians, cross-product face normals;
//   * neighbour face points matched by physical coordinates;
//   * per-element dense mass matrices solved by Cholesky;
//   * the Jacobian-vector product by forward-mode dual numbers;
//   * Jacobian columns by seeding one unknown at a time.
//
// Discrete operator (Section 2.2 names LDG with user-given numerical traces and
// fluxes; the concrete choices are readings documented with the build):
//   q_K:  M_K q_{c,k} = (u_c, d phi/dx_k)_K - <uhat_c n_k, phi>_{dK}
//   R_K:  R_{c,i} = <Fhat_c, phi_i>_{dK} - (f_{c,k}(u,q), d phi_i/dx_k)_K - (s_c, phi_i)_K
//   G(u) = a0 M u - M r + R(u)   (implicit time wrapper; a0 = 0 for steady)
//   uhat = (u- + u+)/2 inside, g on Dirichlet faces, u- otherwise;
//   Fhat = 1/2 (f- + f+).n + sigma (u- - u+) inside, Dirichlet faces use u+ = g, q+ = q-.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

// ----------------------------------------------------------------------------
// Dual numbers (value, tangent) for forward-mode differentiation.
// Non-smooth points: d|x| = sign(x) dx with sign(0) = +1; d max(a,b) takes the
// tangent of a when a >= b.
// ----------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
static inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
static inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
static inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
static inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
static inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
static inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
static inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
static inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
static inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
// Tie convention at the kinks: +1 (default) is the one above; -1 takes the other
// one-sided derivative (sign(0) = -1, the tangent of b when a == b), so that a
// test can form both one-sided directional derivatives at an exact tie.
static int g_tie = 1;
static inline Dual fabs(Dual a) {
  if (a.v > 0) return a;
  if (a.v < 0) return -a;
  return g_tie > 0 ? a : -a;
}
static inline Dual dmax(Dual a, Dual b) {
  if (a.v > b.v) return a;
  if (a.v < b.v) return b;
  return g_tie > 0 ? a : b;
}
static inline double dmax(double a, double b) { return a >= b ? a : b; }
static inline double value(double a) { return a; }
static inline double value(Dual a) { return a.v; }

// ----------------------------------------------------------------------------
// O1: Gauss-Legendre rule on [-1,1] with m points, ascending.
// ----------------------------------------------------------------------------
static void legendre_and_derivative(int m, double x, double& P, double& dP) {
  // three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}
  double p0 = 1.0, p1 = x;
  if (m == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 1; k < m; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1; p1 = p2;
  }
  P = p1;
  dP = m * (x * p1 - p0) / (x * x - 1.0);   // P'_m from P_m, P_{m-1}
}

static void gauss_legendre(int m, std::vector<double>& x, std::vector<double>& w) {
  x.assign(m, 0.0); w.assign(m, 0.0);
  if (m == 1) { x[0] = 0.0; w[0] = 2.0; return; }
  const double pi = std::acos(-1.0);
  for (int i = 0; i < m; ++i) {
    double xi = std::cos(pi * (i + 0.75) / (m + 0.5));   // Chebyshev-like start
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre_and_derivative(m, xi, P, dP);
      double dx = P / dP;
      xi -= dx;
      if (std::fabs(dx) < 1e-15) break;
    }
    double P, dP;
    legendre_and_derivative(m, xi, P, dP);
    x[i] = xi;
    w[i] = 2.0 / ((1.0 - xi * xi) * dP * dP);
  }
  // ascending order
  std::vector<int> idx(m);
  for (int i = 0; i < m; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(m), ws(m);
  for (int i = 0; i < m; ++i) { xs[i] = x[idx[i]]; ws[i] = w[idx[i]]; }
  x = xs; w = ws;
}

// ----------------------------------------------------------------------------
// O2: Lagrange basis by the product formula, derivative by the product rule.
// ----------------------------------------------------------------------------
static double lagrange(const std::vector<double>& nodes, int i, double x) {
  double r = 1.0;
  for (size_t j = 0; j < nodes.size(); ++j)
    if ((int)j != i) r *= (x - nodes[j]) / (nodes[i] - nodes[j]);
  return r;
}
static double dlagrange(const std::vector<double>& nodes, int i, double x) {
  double s = 0.0;
  for (size_t k = 0; k < nodes.size(); ++k) {
    if ((int)k == i) continue;
    double t = 1.0 / (nodes[i] - nodes[k]);
    for (size_t j = 0; j < nodes.size(); ++j)
      if ((int)j != i && j != k) t *= (x - nodes[j]) / (nodes[i] - nodes[j]);
    s += t;
  }
  return s;
}

// ----------------------------------------------------------------------------
// Mesh
// ----------------------------------------------------------------------------
struct OFace {
  long nbr = -1;          // neighbour element, -1 on the boundary
  int nface = -1;         // neighbour's local face
  std::vector<int> perm;  // my face point f  <->  neighbour face point perm[f]
  int tag = -1;           // boundary tag
  long bidx = -1;         // index into the boundary-face list
};

struct OMesh {
  int nd, p, nq, nn, nqv, nqf, nv, nf;
  long E, nbf;
  std::vector<double> X;            // [E][nv][nd] element vertices (periodic images unwrapped)
  std::vector<OFace> faces;         // [E][nf]
  std::vector<double> xn, wn;       // nodes (p+1 GL points) and their weights
  std::vector<double> xq, wq;       // quadrature (nq GL points) and weights
  // volume quadrature data per element: [E][nqv]
  std::vector<double> detJ, Jinv, xv, wv;   // Jinv [E][nqv][nd][nd] = d xi_a / d x_b at [a][b]
  // face quadrature data: [E][nf][nqf]
  std::vector<double> nrm, ds, xf, wf;
  // basis values at volume points [nqv][nn] and derivatives [nqv][nn][nd] (reference)
  std::vector<double> phiV, dphiV;
  // basis values at face points [nf][nqf][nn]
  std::vector<double> phiF;
  std::vector<double> period;
};

// multi-index helpers: flat = i0 + m*i1 + m*m*i2
static void unflat(int flat, int m, int nd, int* ix) {
  for (int k = 0; k < nd; ++k) { ix[k] = flat % m; flat /= m; }
}

// multilinear map and its Jacobian at a reference point
// x(xi) = sum_v N_v(xi) X_v with N_v = prod_k (1 + s_k(v) xi_k) / 2.  Its
// derivative along xi_j is written over the element's edges along j: the edge
// vector (X_hi - X_lo) / 2 weighted by the other directions' shape factors, so
// that a coordinate that does not change along an edge contributes exactly zero
// (axis-aligned faces get exactly axis-aligned normals, which the tie convention
// at |v.n| = 0 relies on).
static void map_point(const OMesh& M, long K, const double* xi, double* x, double* J /*[nd][nd], J[i][j] = dx_i/dxi_j*/) {
  const int nd = M.nd;
  for (int i = 0; i < nd; ++i) { x[i] = 0; for (int j = 0; j < nd; ++j) J[i * nd + j] = 0; }
  for (int v = 0; v < M.nv; ++v) {
    double N = 1.0;
    for (int k = 0; k < nd; ++k) {
      double s = ((v >> k) & 1) ? 1.0 : -1.0;
      N *= 0.5 * (1.0 + s * xi[k]);
    }
    const double* Xv = &M.X[(K * M.nv + v) * nd];
    for (int i = 0; i < nd; ++i) x[i] += N * Xv[i];
  }
  for (int j = 0; j < nd; ++j)
    for (int v = 0; v < M.nv; ++v) {
      if ((v >> j) & 1) continue;                 // edge from corner v to corner v + 2^j
      double w = 0.5;
      for (int k = 0; k < nd; ++k) {
        if (k == j) continue;
        double s = ((v >> k) & 1) ? 1.0 : -1.0;
        w *= 0.5 * (1.0 + s * xi[k]);
      }
      const double* Xlo = &M.X[(K * M.nv + v) * nd];
      const double* Xhi = &M.X[(K * M.nv + (v | (1 << j))) * nd];
      for (int i = 0; i < nd; ++i) J[i * nd + j] += w * (Xhi[i] - Xlo[i]);
    }
}

static double det_and_inverse(int nd, const double* J, double* Ji) {
  if (nd == 1) { Ji[0] = 1.0 / J[0]; return J[0]; }
  if (nd == 2) {
    double d = J[0] * J[3] - J[1] * J[2];
    Ji[0] = J[3] / d; Ji[1] = -J[1] / d; Ji[2] = -J[2] / d; Ji[3] = J[0] / d;
    return d;
  }
  // 3x3 by cofactors
  double c[9];
  c[0] = J[4] * J[8] - J[5] * J[7];
  c[1] = -(J[3] * J[8] - J[5] * J[6]);
  c[2] = J[3] * J[7] - J[4] * J[6];
  c[3] = -(J[1] * J[8] - J[2] * J[7]);
  c[4] = J[0] * J[8] - J[2] * J[6];
  c[5] = -(J[0] * J[7] - J[1] * J[6]);
  c[6] = J[1] * J[5] - J[2] * J[4];
  c[7] = -(J[0] * J[5] - J[2] * J[3]);
  c[8] = J[0] * J[4] - J[1] * J[3];
  double d = J[0] * c[0] + J[1] * c[1] + J[2] * c[2];
  // inverse = adj / det, adj = cof^T
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Ji[a * 3 + b] = c[b * 3 + a] / d;
  return d;
}

// reference coordinates of face point f on local face F
static void face_ref_point(const OMesh& M, int F, int f, double* xi) {
  int dir = F / 2, side = F % 2;
  int t[2], it[2] = {0, 0};
  int nt = 0;
  for (int k = 0; k < M.nd; ++k) if (k != dir) t[nt++] = k;
  int ff = f;
  for (int a = 0; a < nt; ++a) { it[a] = ff % M.nq; ff /= M.nq; }
  xi[dir] = side ? 1.0 : -1.0;
  for (int a = 0; a < nt; ++a) xi[t[a]] = M.xq[it[a]];
}

static OMesh* build_mesh(int nd, int p, int nq, long nvert, const double* vert, long E,
                         const int64_t* ev, const double* period, const int32_t* ftag) {
  if (nd < 1 || nd > 3 || p < 0 || nq < 1) throw std::runtime_error("bad mesh parameters");
  OMesh* Mp = new OMesh();
  OMesh& M = *Mp;
  M.nd = nd; M.p = p; M.nq = nq; M.E = E;
  M.nv = 1 << nd; M.nf = 2 * nd;
  M.nn = 1; M.nqv = 1; M.nqf = 1;
  for (int k = 0; k < nd; ++k) { M.nn *= (p + 1); M.nqv *= nq; }
  for (int k = 0; k < nd - 1; ++k) M.nqf *= nq;
  M.period.assign(period, period + nd);
  gauss_legendre(p + 1, M.xn, M.wn);
  gauss_legendre(nq, M.xq, M.wq);

  // element vertex coordinates with periodic images unwrapped relative to corner 0
  M.X.resize((size_t)E * M.nv * nd);
  for (long K = 0; K < E; ++K) {
    const double* x0 = &vert[ev[K * M.nv] * nd];
    for (int v = 0; v < M.nv; ++v) {
      const double* xv = &vert[ev[K * M.nv + v] * nd];
      for (int k = 0; k < nd; ++k) {
        double c = xv[k];
        if (period[k] > 0) {
          // corner 0 is the low corner: images at exactly half a period go up
          while (c - x0[k] > 0.5 * period[k]) c -= period[k];
          while (x0[k] - c >= 0.5 * period[k]) c += period[k];
        }
        M.X[(K * M.nv + v) * nd + k] = c;
      }
    }
  }

  // basis tables
  M.phiV.assign((size_t)M.nqv * M.nn, 0.0);
  M.dphiV.assign((size_t)M.nqv * M.nn * nd, 0.0);
  int iq[3], in[3];
  for (int q = 0; q < M.nqv; ++q) {
    unflat(q, nq, nd, iq);
    for (int i = 0; i < M.nn; ++i) {
      unflat(i, p + 1, nd, in);
      double v = 1.0;
      for (int k = 0; k < nd; ++k) v *= lagrange(M.xn, in[k], M.xq[iq[k]]);
      M.phiV[(size_t)q * M.nn + i] = v;
      for (int j = 0; j < nd; ++j) {
        double t = 1.0;
        for (int k = 0; k < nd; ++k)
          t *= (k == j) ? dlagrange(M.xn, in[k], M.xq[iq[k]]) : lagrange(M.xn, in[k], M.xq[iq[k]]);
        M.dphiV[((size_t)q * M.nn + i) * nd + j] = t;
      }
    }
  }
  M.phiF.assign((size_t)M.nf * M.nqf * M.nn, 0.0);
  for (int F = 0; F < M.nf; ++F)
    for (int f = 0; f < M.nqf; ++f) {
      double xi[3];
      face_ref_point(M, F, f, xi);
      for (int i = 0; i < M.nn; ++i) {
        unflat(i, p + 1, nd, in);
        double v = 1.0;
        for (int k = 0; k < nd; ++k) v *= lagrange(M.xn, in[k], xi[k]);
        M.phiF[((size_t)F * M.nqf + f) * M.nn + i] = v;
      }
    }

  // volume geometry
  M.detJ.resize((size_t)E * M.nqv);
  M.Jinv.resize((size_t)E * M.nqv * nd * nd);
  M.xv.resize((size_t)E * M.nqv * nd);
  M.wv.resize((size_t)M.nqv);
  for (int q = 0; q < M.nqv; ++q) {
    unflat(q, nq, nd, iq);
    double w = 1.0;
    for (int k = 0; k < nd; ++k) w *= M.wq[iq[k]];
    M.wv[q] = w;
  }
  for (long K = 0; K < E; ++K)
    for (int q = 0; q < M.nqv; ++q) {
      unflat(q, nq, nd, iq);
      double xi[3], x[3], J[9], Ji[9];
      for (int k = 0; k < nd; ++k) xi[k] = M.xq[iq[k]];
      map_point(M, K, xi, x, J);
      double d = det_and_inverse(nd, J, Ji);
      if (!(d > 0)) throw std::runtime_error("element with non-positive Jacobian");
      M.detJ[K * M.nqv + q] = d;
      for (int a = 0; a < nd * nd; ++a) M.Jinv[(K * M.nqv + q) * nd * nd + a] = Ji[a];
      for (int k = 0; k < nd; ++k) M.xv[(K * M.nqv + q) * nd + k] = x[k];
    }

  // face geometry: outward unit normal from the tangent cross product (3D) or the
  // rotated tangent (2D), oriented away from the element centroid.
  M.nrm.resize((size_t)E * M.nf * M.nqf * nd);
  M.ds.resize((size_t)E * M.nf * M.nqf);
  M.xf.resize((size_t)E * M.nf * M.nqf * nd);
  M.wf.resize((size_t)M.nqf);
  for (int f = 0; f < M.nqf; ++f) {
    double w = 1.0; int ff = f;
    for (int a = 0; a < nd - 1; ++a) { w *= M.wq[ff % nq]; ff /= nq; }
    M.wf[f] = w;
  }
  for (long K = 0; K < E; ++K) {
    double xc[3] = {0, 0, 0};
    for (int v = 0; v < M.nv; ++v)
      for (int k = 0; k < nd; ++k) xc[k] += M.X[(K * M.nv + v) * nd + k] / M.nv;
    for (int F = 0; F < M.nf; ++F) {
      int dir = F / 2;
      int t[2], nt = 0;
      for (int k = 0; k < nd; ++k) if (k != dir) t[nt++] = k;
      for (int f = 0; f < M.nqf; ++f) {
        double xi[3], x[3], J[9];
        face_ref_point(M, F, f, xi);
        map_point(M, K, xi, x, J);
        double n[3] = {0, 0, 0};
        if (nd == 1) {
          n[0] = 1.0;
        } else if (nd == 2) {
          double tx = J[0 * 2 + t[0]], ty = J[1 * 2 + t[0]];
          n[0] = ty; n[1] = -tx;
        } else {
          double a[3], b[3];
          for (int i = 0; i < 3; ++i) { a[i] = J[i * 3 + t[0]]; b[i] = J[i * 3 + t[1]]; }
          n[0] = a[1] * b[2] - a[2] * b[1];
          n[1] = a[2] * b[0] - a[0] * b[2];
          n[2] = a[0] * b[1] - a[1] * b[0];
        }
        double dot = 0, nn = 0;
        for (int k = 0; k < nd; ++k) { dot += n[k] * (x[k] - xc[k]); nn += n[k] * n[k]; }
        nn = std::sqrt(nn);
        double s = dot >= 0 ? 1.0 : -1.0;
        size_t o = ((size_t)K * M.nf + F) * M.nqf + f;
        M.ds[o] = nn;
        for (int k = 0; k < nd; ++k) { M.nrm[o * nd + k] = s * n[k] / nn; M.xf[o * nd + k] = x[k]; }
      }
    }
  }

  // connectivity: faces keyed by their sorted corner vertex ids; matched face
  // points found by physical coordinates modulo the period.
  M.faces.assign((size_t)E * M.nf, OFace());
  std::map<std::vector<int64_t>, std::vector<std::pair<long, int>>> fmap;
  for (long K = 0; K < E; ++K)
    for (int F = 0; F < M.nf; ++F) {
      int dir = F / 2, side = F % 2;
      std::vector<int64_t> key;
      for (int v = 0; v < M.nv; ++v)
        if (((v >> dir) & 1) == side) key.push_back(ev[K * M.nv + v]);
      std::sort(key.begin(), key.end());
      fmap[key].push_back({K, F});
    }
  double scale = 0;
  for (long i = 0; i < nvert * nd; ++i) scale = std::max(scale, std::fabs(vert[i]));
  scale = std::max(scale, 1.0);
  for (auto& kv : fmap) {
    auto& lst = kv.second;
    if (lst.size() > 2) throw std::runtime_error("face shared by more than two elements");
    if (lst.size() == 2) {
      for (int s = 0; s < 2; ++s) {
        long K = lst[s].first; int F = lst[s].second;
        long K2 = lst[1 - s].first; int F2 = lst[1 - s].second;
        OFace& fc = M.faces[(size_t)K * M.nf + F];
        fc.nbr = K2; fc.nface = F2; fc.perm.assign(M.nqf, -1);
        for (int f = 0; f < M.nqf; ++f) {
          const double* xa = &M.xf[(((size_t)K * M.nf + F) * M.nqf + f) * nd];
          int found = -1;
          for (int g = 0; g < M.nqf; ++g) {
            const double* xb = &M.xf[(((size_t)K2 * M.nf + F2) * M.nqf + g) * nd];
            double err = 0;
            for (int k = 0; k < nd; ++k) {
              double dlt = xa[k] - xb[k];
              if (M.period[k] > 0) dlt -= M.period[k] * std::round(dlt / M.period[k]);
              err = std::max(err, std::fabs(dlt));
            }
            if (err <= 1e-12 * scale) { found = g; break; }
          }
          if (found < 0) throw std::runtime_error("neighbour face points do not match");
          fc.perm[f] = found;
        }
      }
    }
  }
  // boundary faces in element-major, local-face-minor order
  M.nbf = 0;
  for (long K = 0; K < E; ++K)
    for (int F = 0; F < M.nf; ++F) {
      OFace& fc = M.faces[(size_t)K * M.nf + F];
      if (fc.nbr < 0) {
        fc.bidx = M.nbf++;
        fc.tag = ftag ? ftag[K * M.nf + F] : 0;
        if (fc.tag < 0) fc.tag = 0;
      }
    }
  return Mp;
}

// ----------------------------------------------------------------------------
// Models: pointwise flux f(u,q) [ncu][nd], source s, numerical flux.
// kind 0: Poisson/heat      f = kappa q,                 s = src - lambda u
// kind 1: convection-diff.  f = kappa q + b u,           s = src
// kind 2: Euler             f = inviscid flux,           s = src
// kind 3: Navier-Stokes     f = inviscid - viscous(u, grad u = -q)
// kind 4: shallow water     f = (h v, h v v^T + g h^2/2 I), g = mu[0]
// kind 5: wave (first order) state (u, q): f = (c^2 q, u I), c^2 = mu[0]
// mu: Poisson [kappa0, tau, lambda]; conv-diff [kappa0, tau];
//     Euler [gamma]; NS [gamma, Re, Pr, tau]
// aux (nodal): Poisson [kappa-factor]; conv-diff [kappa, b_1..b_nd]
// ----------------------------------------------------------------------------
struct OModel {
  int kind, ncu, naux, nd;
  std::vector<double> mu;
  const double* aux;   // [E][naux][nn]
  const double* src;   // [E][ncu][nqv]
  const double* bdata; // [nbf][ncu][nqf]
  std::vector<int> bc_kind;   // per tag: 0 Dirichlet, 1 Neumann (flux data), 2 extrapolation, 3 slip wall
  double a0;
  const double* r;     // [E][ncu][nn] or null
};

static double mu_or(const OModel& md, int i, double def) {
  return (int)md.mu.size() > i ? md.mu[i] : def;
}

template <class T>
static void phys_flux(const OModel& md, const T* u, const T* q, const double* a, T* f) {
  const int nd = md.nd;
  if (md.kind == 0) {
    double kap = mu_or(md, 0, 1.0) * (md.naux >= 1 ? a[0] : 1.0);
    for (int k = 0; k < nd; ++k) f[k] = kap * q[k];
  } else if (md.kind == 1) {
    double kap = mu_or(md, 0, 1.0) * a[0];
    for (int k = 0; k < nd; ++k) f[k] = kap * q[k] + a[1 + k] * u[0];
  } else if (md.kind == 5) {
    // wave model as a first-order system, state (u, q): u_t + div(c^2 q) = 0, q_t + grad u = 0,
    // i.e. f = (c^2 q, u I), c^2 = mu[0]
    const double c2 = mu_or(md, 0, 1.0);
    for (int k = 0; k < nd; ++k) {
      f[0 * nd + k] = c2 * u[1 + k];
      for (int i = 0; i < nd; ++i) f[(1 + i) * nd + k] = (i == k) ? u[0] : T(0.0);
    }
  } else if (md.kind == 4) {
    // shallow water, u = (h, h v): f = (h v, h v v^T + g h^2 / 2 I), g = mu[0]
    const double g = mu_or(md, 0, 1.0);
    T h = u[0];
    T half_gh2 = 0.5 * g * h * h;
    for (int k = 0; k < nd; ++k) {
      f[0 * nd + k] = u[1 + k];
      for (int i = 0; i < nd; ++i) f[(1 + i) * nd + k] = u[1 + i] * u[1 + k] / h + (i == k ? half_gh2 : T(0.0));
    }
  } else {
    const double gam = mu_or(md, 0, 1.4);
    const int ne = nd + 1;
    T rho = u[0], E = u[ne];
    T vel[3], ke = T(0.0);
    for (int k = 0; k < nd; ++k) { vel[k] = u[1 + k] / rho; ke += u[1 + k] * vel[k]; }
    T pr = (gam - 1.0) * (E - 0.5 * ke);
    for (int k = 0; k < nd; ++k) {
      f[0 * nd + k] = u[1 + k];
      for (int i = 0; i < nd; ++i) f[(1 + i) * nd + k] = u[1 + i] * vel[k] + (i == k ? pr : T(0.0));
      f[ne * nd + k] = (E + pr) * vel[k];
    }
    if (md.kind == 3) {
      const double Re = mu_or(md, 1, 1.0), Pr = mu_or(md, 2, 0.72);
      const double vis = 1.0 / Re;
      // gradients of the conservative variables: grad u = -q
      T gr[3], gm[3][3], gE[3];
      for (int k = 0; k < nd; ++k) {
        gr[k] = -q[0 * nd + k];
        for (int i = 0; i < nd; ++i) gm[i][k] = -q[(1 + i) * nd + k];
        gE[k] = -q[ne * nd + k];
      }
      T gv[3][3], ge[3];
      T Em = E / rho;
      for (int k = 0; k < nd; ++k) {
        for (int i = 0; i < nd; ++i) gv[i][k] = (gm[i][k] - vel[i] * gr[k]) / rho;
        T gEm = (gE[k] - Em * gr[k]) / rho;
        T s = gEm;
        for (int i = 0; i < nd; ++i) s -= vel[i] * gv[i][k];
        ge[k] = s;
      }
      T divv = T(0.0);
      for (int i = 0; i < nd; ++i) divv += gv[i][i];
      for (int k = 0; k < nd; ++k) {
        T work = T(0.0);
        for (int i = 0; i < nd; ++i) {
          T tau = vis * (gv[i][k] + gv[k][i]);
          if (i == k) tau -= vis * (2.0 / 3.0) * divv;
          f[(1 + i) * nd + k] -= tau;
          work += vel[i] * tau;
        }
        f[ne * nd + k] -= work + vis * gam / Pr * ge[k];
      }
    }
  }
}

// max wave speed |v.n| + c for the Euler/NS Lax-Friedrichs flux
template <class T>
static T wave_speed(const OModel& md, const T* u, const double* n) {
  const int nd = md.nd;
  if (md.kind == 5) return T(std::sqrt(mu_or(md, 0, 1.0)));   // wave speed c
  if (md.kind == 4) {
    // shallow water: |v.n| + sqrt(g h)
    T vn = T(0.0);
    for (int k = 0; k < nd; ++k) vn += u[1 + k] / u[0] * n[k];
    return fabs(vn) + sqrt(mu_or(md, 0, 1.0) * u[0]);
  }
  const double gam = mu_or(md, 0, 1.4);
  T rho = u[0], E = u[nd + 1];
  T vn = T(0.0), ke = T(0.0);
  for (int k = 0; k < nd; ++k) { vn += u[1 + k] / rho * n[k]; ke += u[1 + k] * u[1 + k] / rho; }
  T pr = (gam - 1.0) * (E - 0.5 * ke);
  return fabs(vn) + sqrt(gam * pr / rho);
}

// interior (or Dirichlet with u+ = g, q+ = q-) numerical flux, n = outward normal of the minus side
template <class T>
static void num_flux(const OModel& md, const T* uL, const T* qL, const double* aL,
                     const T* uR, const T* qR, const double* aR, const double* n, T* Fh) {
  const int nd = md.nd, ncu = md.ncu;
  T fL[5 * 3], fR[5 * 3];
  phys_flux(md, uL, qL, aL, fL);
  phys_flux(md, uR, qR, aR, fR);
  for (int c = 0; c < ncu; ++c) {
    T s = T(0.0);
    for (int k = 0; k < nd; ++k) s += 0.5 * (fL[c * nd + k] + fR[c * nd + k]) * n[k];
    Fh[c] = s;
  }
  if (md.kind == 0) {
    double kL = md.naux >= 1 ? aL[0] : 1.0, kR = md.naux >= 1 ? aR[0] : 1.0;
    double sig = mu_or(md, 1, 1.0) * mu_or(md, 0, 1.0) * 0.5 * (kL + kR);
    Fh[0] += sig * (uL[0] - uR[0]);
  } else if (md.kind == 1) {
    double sig = mu_or(md, 1, 1.0) * mu_or(md, 0, 1.0) * 0.5 * (aL[0] + aR[0]);
    double bnL = 0, bnR = 0;
    for (int k = 0; k < nd; ++k) { bnL += aL[1 + k] * n[k]; bnR += aR[1 + k] * n[k]; }
    sig += 0.5 * dmax(std::fabs(bnL), std::fabs(bnR));
    Fh[0] += sig * (uL[0] - uR[0]);
  } else {
    T lam = dmax(wave_speed(md, uL, n), wave_speed(md, uR, n));
    T sig = 0.5 * lam;
    if (md.kind == 3) sig += mu_or(md, 3, 1.0) / mu_or(md, 1, 1.0);
    for (int c = 0; c < ncu; ++c) Fh[c] += sig * (uL[c] - uR[c]);
  }
}

// ----------------------------------------------------------------------------
// Element-level pieces of the operator
// ----------------------------------------------------------------------------
template <class T>
struct OState {
  const OMesh* M;
  const OModel* md;
  const T* u;                 // [E][ncu][nn]
  std::vector<T> q;           // [E][ncu][nd][nn]
  std::vector<char> have_q;
};

// aux at an arbitrary point given nodal basis values phi[nn]
static void aux_at(const OMesh& M, const OModel& md, long K, const double* phi, double* a) {
  for (int j = 0; j < md.naux; ++j) {
    double s = 0;
    for (int i = 0; i < M.nn; ++i) s += md.aux[((size_t)K * md.naux + j) * M.nn + i] * phi[i];
    a[j] = s;
  }
}

template <class T>
static void trace_u(const OMesh& M, const OModel& md, const T* u, long K, int F, int f, T* out) {
  const double* phi = &M.phiF[((size_t)F * M.nqf + f) * M.nn];
  for (int c = 0; c < md.ncu; ++c) {
    T s = T(0.0);
    for (int i = 0; i < M.nn; ++i) s += u[((size_t)K * md.ncu + c) * M.nn + i] * phi[i];
    out[c] = s;
  }
}

template <class T>
static void trace_q(const OMesh& M, const OModel& md, const T* q, long K, int F, int f, T* out) {
  const double* phi = &M.phiF[((size_t)F * M.nqf + f) * M.nn];
  for (int c = 0; c < md.ncu; ++c)
    for (int k = 0; k < M.nd; ++k) {
      T s = T(0.0);
      for (int i = 0; i < M.nn; ++i) s += q[(((size_t)K * md.ncu + c) * M.nd + k) * M.nn + i] * phi[i];
      out[c * M.nd + k] = s;
    }
}

// Cholesky solve of the SPD element mass matrix, one right-hand side at a time
static void cholesky(int n, std::vector<double>& A) {
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
    if (!(s > 0)) throw std::runtime_error("mass matrix not SPD");
    A[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = t / A[j * n + j];
    }
  }
}
template <class T>
static void cholesky_solve(int n, const std::vector<double>& L, T* b) {
  for (int i = 0; i < n; ++i) {
    T s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
    b[i] = s / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    T s = b[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
    b[i] = s / L[i * n + i];
  }
}

static std::vector<double> mass_matrix(const OMesh& M, long K) {
  std::vector<double> A((size_t)M.nn * M.nn, 0.0);
  for (int q = 0; q < M.nqv; ++q) {
    double wj = M.wv[q] * M.detJ[K * M.nqv + q];
    const double* phi = &M.phiV[(size_t)q * M.nn];
    for (int i = 0; i < M.nn; ++i)
      for (int j = 0; j < M.nn; ++j) A[i * M.nn + j] += wj * phi[i] * phi[j];
  }
  return A;
}

// physical gradient of basis function i at volume point q of element K
static void grad_phi(const OMesh& M, long K, int q, int i, double* g) {
  const int nd = M.nd;
  const double* dphi = &M.dphiV[((size_t)q * M.nn + i) * nd];
  const double* Ji = &M.Jinv[((size_t)K * M.nqv + q) * nd * nd];
  for (int k = 0; k < nd; ++k) {
    double s = 0;
    for (int a = 0; a < nd; ++a) s += dphi[a] * Ji[a * nd + k];   // d phi/d x_k = sum_a d phi/d xi_a * d xi_a/d x_k
    g[k] = s;
  }
}

// numerical trace uhat at face point f of face F of K (ncu values)
template <class T>
static void uhat_at(const OMesh& M, const OModel& md, const T* u, long K, int F, int f, T* uh) {
  const OFace& fc = M.faces[(size_t)K * M.nf + F];
  T um[5];
  trace_u(M, md, u, K, F, f, um);
  if (fc.nbr >= 0) {
    T up[5];
    trace_u(M, md, u, fc.nbr, fc.nface, fc.perm[f], up);
    for (int c = 0; c < md.ncu; ++c) uh[c] = 0.5 * (um[c] + up[c]);
  } else {
    int kind = md.bc_kind.empty() ? 0 : md.bc_kind[std::min<int>(fc.tag, (int)md.bc_kind.size() - 1)];
    if (kind == 0) {
      for (int c = 0; c < md.ncu; ++c) uh[c] = T(md.bdata ? md.bdata[((size_t)fc.bidx * md.ncu + c) * M.nqf + f] : 0.0);
    } else {
      for (int c = 0; c < md.ncu; ++c) uh[c] = um[c];
    }
  }
}

// O5: the LDG gradient q of element K (Eq. 1a in weak form)
template <class T>
static void compute_q(const OMesh& M, const OModel& md, const T* u, long K, T* qK /*[ncu][nd][nn]*/) {
  const int nd = M.nd, nn = M.nn, ncu = md.ncu;
  std::vector<T> b((size_t)ncu * nd * nn, T(0.0));
  for (int q = 0; q < M.nqv; ++q) {
    double wj = M.wv[q] * M.detJ[K * M.nqv + q];
    const double* phi = &M.phiV[(size_t)q * nn];
    for (int c = 0; c < ncu; ++c) {
      T uq = T(0.0);
      for (int j = 0; j < nn; ++j) uq += u[((size_t)K * ncu + c) * nn + j] * phi[j];
      for (int i = 0; i < nn; ++i) {
        double g[3];
        grad_phi(M, K, q, i, g);
        for (int k = 0; k < nd; ++k) b[((size_t)c * nd + k) * nn + i] += wj * g[k] * uq;
      }
    }
  }
  for (int F = 0; F < M.nf; ++F)
    for (int f = 0; f < M.nqf; ++f) {
      size_t o = ((size_t)K * M.nf + F) * M.nqf + f;
      double wds = M.wf[f] * M.ds[o];
      const double* n = &M.nrm[o * nd];
      const double* phi = &M.phiF[((size_t)F * M.nqf + f) * nn];
      T uh[5];
      uhat_at(M, md, u, K, F, f, uh);
      for (int c = 0; c < ncu; ++c)
        for (int k = 0; k < nd; ++k)
          for (int i = 0; i < nn; ++i) b[((size_t)c * nd + k) * nn + i] -= wds * n[k] * phi[i] * uh[c];
    }
  std::vector<double> L = mass_matrix(M, K);
  cholesky(nn, L);
  for (int c = 0; c < ncu; ++c)
    for (int k = 0; k < nd; ++k) cholesky_solve(nn, L, &b[((size_t)c * nd + k) * nn]);
  for (size_t i = 0; i < b.size(); ++i) qK[i] = b[i];
}

static bool model_has_q(const OModel& md) { return md.kind <= 1 || md.kind == 3; }

// O6 + O7: residual G_K of element K given q on K and on its face neighbours
template <class T>
static void element_residual(const OMesh& M, const OModel& md, const T* u, const T* q, long K, T* RK) {
  const int nd = M.nd, nn = M.nn, ncu = md.ncu;
  for (int i = 0; i < ncu * nn; ++i) RK[i] = T(0.0);
  const bool hq = model_has_q(md);
  T zq[15];
  for (int i = 0; i < 15; ++i) zq[i] = T(0.0);
  // volume: - (f, grad phi_i) - (s, phi_i)
  for (int qp = 0; qp < M.nqv; ++qp) {
    double wj = M.wv[qp] * M.detJ[K * M.nqv + qp];
    const double* phi = &M.phiV[(size_t)qp * nn];
    T uq[5], qq[15];
    for (int c = 0; c < ncu; ++c) {
      T s = T(0.0);
      for (int j = 0; j < nn; ++j) s += u[((size_t)K * ncu + c) * nn + j] * phi[j];
      uq[c] = s;
      for (int k = 0; k < nd; ++k) {
        T t = T(0.0);
        if (hq)
          for (int j = 0; j < nn; ++j) t += q[(((size_t)K * ncu + c) * nd + k) * nn + j] * phi[j];
        qq[c * nd + k] = t;
      }
    }
    double a[4] = {0, 0, 0, 0};
    aux_at(M, md, K, phi, a);
    T f[15];
    phys_flux(md, uq, qq, a, f);
    T s[5];
    for (int c = 0; c < ncu; ++c) {
      s[c] = T(md.src ? md.src[((size_t)K * ncu + c) * M.nqv + qp] : 0.0);
      if (md.kind == 0) s[c] -= mu_or(md, 2, 0.0) * uq[c];
    }
    for (int i = 0; i < nn; ++i) {
      double g[3];
      grad_phi(M, K, qp, i, g);
      for (int c = 0; c < ncu; ++c) {
        T t = s[c] * phi[i];
        for (int k = 0; k < nd; ++k) t += f[c * nd + k] * g[k];
        RK[c * nn + i] -= wj * t;
      }
    }
  }
  // faces: + <Fhat, phi_i>
  for (int F = 0; F < M.nf; ++F) {
    const OFace& fc = M.faces[(size_t)K * M.nf + F];
    for (int f = 0; f < M.nqf; ++f) {
      size_t o = ((size_t)K * M.nf + F) * M.nqf + f;
      double wds = M.wf[f] * M.ds[o];
      const double* n = &M.nrm[o * nd];
      const double* phi = &M.phiF[((size_t)F * M.nqf + f) * nn];
      T um[5], qm[15], Fh[5];
      trace_u(M, md, u, K, F, f, um);
      if (hq) trace_q(M, md, q, K, F, f, qm); else for (int i = 0; i < 15; ++i) qm[i] = zq[i];
      double am[4] = {0, 0, 0, 0};
      aux_at(M, md, K, phi, am);
      if (fc.nbr >= 0) {
        T up[5], qp[15];
        int g = fc.perm[f];
        trace_u(M, md, u, fc.nbr, fc.nface, g, up);
        if (hq) trace_q(M, md, q, fc.nbr, fc.nface, g, qp); else for (int i = 0; i < 15; ++i) qp[i] = zq[i];
        double ap[4] = {0, 0, 0, 0};
        aux_at(M, md, fc.nbr, &M.phiF[((size_t)fc.nface * M.nqf + g) * nn], ap);
        num_flux(md, um, qm, am, up, qp, ap, n, Fh);
      } else {
        int kind = md.bc_kind.empty() ? 0 : md.bc_kind[std::min<int>(fc.tag, (int)md.bc_kind.size() - 1)];
        if (kind == 0) {
          T ub[5];
          for (int c = 0; c < ncu; ++c) ub[c] = T(md.bdata ? md.bdata[((size_t)fc.bidx * ncu + c) * M.nqf + f] : 0.0);
          num_flux(md, um, qm, am, ub, qm, am, n, Fh);
        } else if (kind == 1) {
          for (int c = 0; c < ncu; ++c) Fh[c] = T(md.bdata ? md.bdata[((size_t)fc.bidx * ncu + c) * M.nqf + f] : 0.0);
        } else if (kind == 3) {
          // slip wall (Euler, shallow water): the outside state is the inside one with its normal
          // momentum reversed, so the wall passes no mass and no energy
          T ub[5], mn = T(0.0);
          for (int k = 0; k < nd; ++k) mn += um[1 + k] * n[k];
          for (int c = 0; c < ncu; ++c) ub[c] = um[c];
          for (int k = 0; k < nd; ++k) ub[1 + k] = um[1 + k] - 2.0 * mn * n[k];
          num_flux(md, um, qm, am, ub, qm, am, n, Fh);
        } else {
          T fl[15];
          phys_flux(md, um, qm, am, fl);
          for (int c = 0; c < ncu; ++c) {
            T s = T(0.0);
            for (int k = 0; k < nd; ++k) s += fl[c * nd + k] * n[k];
            Fh[c] = s;
          }
        }
      }
      for (int c = 0; c < ncu; ++c)
        for (int i = 0; i < nn; ++i) RK[c * nn + i] += wds * Fh[c] * phi[i];
    }
  }
  // time wrapper: + a0 M u - M r
  if (md.a0 != 0.0 || md.r) {
    std::vector<double> Mm = mass_matrix(M, K);
    for (int c = 0; c < ncu; ++c)
      for (int i = 0; i < nn; ++i) {
        T s = T(0.0);
        for (int j = 0; j < nn; ++j) {
          T t = md.a0 * u[((size_t)K * ncu + c) * nn + j];
          if (md.r) t -= md.r[((size_t)K * ncu + c) * nn + j];
          s += Mm[i * nn + j] * t;
        }
        RK[c * nn + i] += s;
      }
  }
}

template <class T>
static void full_residual(const OMesh& M, const OModel& md, const T* u, T* R, T* qout) {
  const size_t nq = (size_t)M.E * md.ncu * M.nd * M.nn;
  std::vector<T> q(model_has_q(md) ? nq : 1, T(0.0));
  if (model_has_q(md))
    for (long K = 0; K < M.E; ++K) compute_q(M, md, u, K, &q[(size_t)K * md.ncu * M.nd * M.nn]);
  for (long K = 0; K < M.E; ++K) element_residual(M, md, u, q.data(), K, &R[(size_t)K * md.ncu * M.nn]);
  if (qout && model_has_q(md))
    for (size_t i = 0; i < nq; ++i) qout[i] = q[i];
}

// elements within face-graph distance <= depth of K
static std::vector<long> neighbourhood(const OMesh& M, long K, int depth) {
  std::vector<long> cur{K}, all{K};
  for (int d = 0; d < depth; ++d) {
    std::vector<long> nxt;
    for (long e : cur)
      for (int F = 0; F < M.nf; ++F) {
        long nb = M.faces[(size_t)e * M.nf + F].nbr;
        if (nb >= 0 && std::find(all.begin(), all.end(), nb) == all.end()) { all.push_back(nb); nxt.push_back(nb); }
      }
    cur = nxt;
  }
  return all;
}

// ----------------------------------------------------------------------------
// C ABI (host pointers)
// ----------------------------------------------------------------------------
static thread_local std::string g_err;

struct ldgo_model_desc {
  int kind, ncu, nmu;
  const double* mu;
  int naux;
  const double* aux;
  const double* src;
  const double* bdata;
  int nbc;
  const int* bc_kind;
  double a0;
  const double* r;
};

static OModel to_model(const OMesh& M, const ldgo_model_desc* d) {
  OModel md;
  md.kind = d->kind; md.ncu = d->ncu; md.naux = d->naux; md.nd = M.nd;
  md.mu.assign(d->mu, d->mu + d->nmu);
  md.aux = d->aux; md.src = d->src; md.bdata = d->bdata;
  md.bc_kind.assign(d->bc_kind, d->bc_kind + d->nbc);
  md.a0 = d->a0; md.r = d->r;
  if (md.kind < 0 || md.kind > 5) throw std::runtime_error("unknown model");
  if ((md.kind <= 1 && md.ncu != 1) || ((md.kind == 2 || md.kind == 3) && md.ncu != M.nd + 2) ||
      ((md.kind == 4 || md.kind == 5) && md.ncu != M.nd + 1))
    throw std::runtime_error("ncu inconsistent with the model");
  if (md.kind == 1 && md.naux != 1 + M.nd) throw std::runtime_error("convection-diffusion needs aux = [kappa, b]");
  for (int b : md.bc_kind) {
    if (b < 0 || b > 3) throw std::runtime_error("unknown boundary kind");
    if (b == 3 && md.kind != 2 && md.kind != 4) throw std::runtime_error("slip walls need Euler or shallow water");
  }
  return md;
}

#define GUARD(...) try { __VA_ARGS__; return 0; } catch (const std::exception& e) { g_err = e.what(); return -1; }

extern "C" {

const char* ldgo_last_error() { return g_err.c_str(); }

// +1: sign(0) = +1 and max ties take the first argument's tangent (the default);
// -1: the opposite one-sided choice.  Returns the previous setting.
int ldgo_set_tie_break(int t) {
  const int old = g_tie;
  g_tie = t >= 0 ? 1 : -1;
  return old;
}

int ldgo_gauss_legendre(int m, double* x, double* w) {
  GUARD({ std::vector<double> a, b; gauss_legendre(m, a, b); for (int i = 0; i < m; ++i) { x[i] = a[i]; w[i] = b[i]; } })
}

double ldgo_lagrange(int n, const double* nodes, int i, double x, int deriv) {
  std::vector<double> nd(nodes, nodes + n);
  return deriv ? dlagrange(nd, i, x) : lagrange(nd, i, x);
}

void* ldgo_mesh_create(int nd, int p, int nq, int64_t nvert, const double* vert, int64_t E,
                       const int64_t* elem_vert, const double* period, const int32_t* face_tag) {
  try { return build_mesh(nd, p, nq, nvert, vert, E, elem_vert, period, face_tag); }
  catch (const std::exception& e) { g_err = e.what(); return nullptr; }
}

void ldgo_mesh_destroy(void* h) { delete (OMesh*)h; }

// out: [E, nn, nqv, nqf, nbf]
void ldgo_mesh_info(void* h, int64_t* out) {
  OMesh& M = *(OMesh*)h;
  out[0] = M.E; out[1] = M.nn; out[2] = M.nqv; out[3] = M.nqf; out[4] = M.nbf;
}

// node coordinates [E][nn][nd], volume quadrature points [E][nqv][nd],
// boundary face quadrature points [nbf][nqf][nd], boundary face (element, face) [nbf][2]
void ldgo_mesh_points(void* h, double* xnode, double* xquad, double* xbf, int64_t* bf) {
  OMesh& M = *(OMesh*)h;
  const int nd = M.nd;
  if (xnode) {
    int in[3];
    for (long K = 0; K < M.E; ++K)
      for (int i = 0; i < M.nn; ++i) {
        unflat(i, M.p + 1, nd, in);
        double xi[3], x[3], J[9];
        for (int k = 0; k < nd; ++k) xi[k] = M.xn[in[k]];
        map_point(M, K, xi, x, J);
        for (int k = 0; k < nd; ++k) xnode[((size_t)K * M.nn + i) * nd + k] = x[k];
      }
  }
  if (xquad) std::memcpy(xquad, M.xv.data(), M.xv.size() * sizeof(double));
  for (long K = 0; K < M.E; ++K)
    for (int F = 0; F < M.nf; ++F) {
      const OFace& fc = M.faces[(size_t)K * M.nf + F];
      if (fc.nbr >= 0) continue;
      if (bf) { bf[fc.bidx * 2] = K; bf[fc.bidx * 2 + 1] = F; }
      if (xbf)
        for (int f = 0; f < M.nqf; ++f)
          for (int k = 0; k < nd; ++k)
            xbf[((size_t)fc.bidx * M.nqf + f) * nd + k] = M.xf[(((size_t)K * M.nf + F) * M.nqf + f) * nd + k];
    }
}

// per element: volume (sum of w |J|) and the closed-surface integral of n ds [E][nd]
void ldgo_mesh_geometry_checks(void* h, double* vol, double* nsum) {
  OMesh& M = *(OMesh*)h;
  for (long K = 0; K < M.E; ++K) {
    double v = 0;
    for (int q = 0; q < M.nqv; ++q) v += M.wv[q] * M.detJ[K * M.nqv + q];
    vol[K] = v;
    for (int k = 0; k < M.nd; ++k) {
      double s = 0;
      for (int F = 0; F < M.nf; ++F)
        for (int f = 0; f < M.nqf; ++f) {
          size_t o = ((size_t)K * M.nf + F) * M.nqf + f;
          s += M.wf[f] * M.ds[o] * M.nrm[o * M.nd + k];
        }
      nsum[K * M.nd + k] = s;
    }
  }
}

// neighbour table [E][2nd] (-1 on the boundary), for tests of connectivity
void ldgo_mesh_neighbours(void* h, int64_t* nbr) {
  OMesh& M = *(OMesh*)h;
  for (long K = 0; K < M.E; ++K)
    for (int F = 0; F < M.nf; ++F) nbr[K * M.nf + F] = M.faces[(size_t)K * M.nf + F].nbr;
}

// G(u) and optionally q(u)
int ldgo_residual(void* h, const ldgo_model_desc* d, const double* u, double* R, double* q) {
  GUARD({
    OMesh& M = *(OMesh*)h;
    OModel md = to_model(M, d);
    full_residual<double>(M, md, u, R, q);
  })
}

// J(u) v by forward-mode dual numbers; optionally the tangent of q
int ldgo_jvp(void* h, const ldgo_model_desc* d, const double* u, const double* v, double* Jv, double* dq) {
  GUARD({
    OMesh& M = *(OMesh*)h;
    OModel md = to_model(M, d);
    size_t N = (size_t)M.E * md.ncu * M.nn;
    std::vector<Dual> ud(N), Rd(N);
    for (size_t i = 0; i < N; ++i) ud[i] = Dual(u[i], v[i]);
    size_t nq = (size_t)M.E * md.ncu * M.nd * M.nn;
    std::vector<Dual> qd(model_has_q(md) ? nq : 1);
    full_residual<Dual>(M, md, ud.data(), Rd.data(), qd.data());
    for (size_t i = 0; i < N; ++i) Jv[i] = Rd[i].d;
    if (dq && model_has_q(md)) for (size_t i = 0; i < nq; ++i) dq[i] = qd[i].d;
  })
}

// All columns of the Jacobian dG/du, each by a dual pass seeded at one unknown
// and restricted to the elements whose residual can depend on it (face-graph
// distance <= 2; their q needs distance <= 3).  COO output; returns nnz or -1.
int64_t ldgo_jacobian_coo(void* h, const ldgo_model_desc* d, const double* u, int64_t cap,
                          int64_t* rows, int64_t* cols, double* vals) {
  try {
    OMesh& M = *(OMesh*)h;
    OModel md = to_model(M, d);
    const int ncu = md.ncu, nn = M.nn, nd = M.nd;
    const size_t N = (size_t)M.E * ncu * nn;
    std::vector<Dual> ud(N);
    for (size_t i = 0; i < N; ++i) ud[i] = Dual(u[i], 0.0);
    const size_t qsz = (size_t)ncu * nd * nn;
    std::vector<Dual> q(model_has_q(md) ? (size_t)M.E * qsz : 1);
    std::vector<Dual> RK((size_t)ncu * nn);
    int64_t nnz = 0;
    for (long K0 = 0; K0 < M.E; ++K0) {
      std::vector<long> S2 = neighbourhood(M, K0, 2);
      std::vector<long> S3 = model_has_q(md) ? neighbourhood(M, K0, 3) : std::vector<long>();
      for (int j = 0; j < ncu * nn; ++j) {
        size_t col = (size_t)K0 * ncu * nn + j;
        ud[col].d = 1.0;
        for (long e : S3) compute_q(M, md, ud.data(), e, &q[(size_t)e * qsz]);
        for (long e : S2) {
          element_residual(M, md, ud.data(), q.data(), e, RK.data());
          for (int i = 0; i < ncu * nn; ++i) {
            if (RK[i].d == 0.0) continue;
            if (nnz >= cap) throw std::runtime_error("jacobian capacity exceeded");
            rows[nnz] = (int64_t)e * ncu * nn + i; cols[nnz] = (int64_t)col; vals[nnz] = RK[i].d; ++nnz;
          }
        }
        ud[col].d = 0.0;
      }
    }
    return nnz;
  } catch (const std::exception& e) { g_err = e.what(); return -1; }
}

// Diagonal blocks dG_K/du_K for the listed elements: [nsel][nb][nb] row-major,
// nb = ncu*nn (per_variable=0) or [nsel][ncu][nn][nn] (per_variable=1).
int ldgo_jacobian_blocks(void* h, const ldgo_model_desc* d, const double* u, int64_t nsel,
                         const int64_t* sel, int per_variable, double* blocks) {
  GUARD({
    OMesh& M = *(OMesh*)h;
    OModel md = to_model(M, d);
    const int ncu = md.ncu, nn = M.nn, nd = M.nd, nb = ncu * nn;
    const size_t N = (size_t)M.E * nb;
    std::vector<Dual> ud(N);
    for (size_t i = 0; i < N; ++i) ud[i] = Dual(u[i], 0.0);
    const size_t qsz = (size_t)ncu * nd * nn;
    std::vector<Dual> q(model_has_q(md) ? (size_t)M.E * qsz : 1);
    std::vector<Dual> RK(nb);
    for (int64_t s = 0; s < nsel; ++s) {
      long K = sel[s];
      std::vector<long> S1 = model_has_q(md) ? neighbourhood(M, K, 1) : std::vector<long>();
      for (int j = 0; j < nb; ++j) {
        size_t col = (size_t)K * nb + j;
        ud[col].d = 1.0;
        for (long e : S1) compute_q(M, md, ud.data(), e, &q[(size_t)e * qsz]);
        element_residual(M, md, ud.data(), q.data(), K, RK.data());
        for (int i = 0; i < nb; ++i) {
          if (per_variable) {
            int ci = i / nn, cj = j / nn;
            if (ci == cj) blocks[(((size_t)s * ncu + ci) * nn + (i % nn)) * nn + (j % nn)] = RK[i].d;
          } else {
            blocks[((size_t)s * nb + i) * nb + j] = RK[i].d;
          }
        }
        ud[col].d = 0.0;
      }
    }
  })
}

// G_K and (J v)_K for the listed elements only (q computed on each element and
// its face neighbours): lets large meshes be checked on a sample of elements.
int ldgo_sample_elements(void* h, const ldgo_model_desc* d, const double* u, const double* v, int64_t nsel,
                         const int64_t* sel, double* G, double* Jv) {
  GUARD({
    OMesh& M = *(OMesh*)h;
    OModel md = to_model(M, d);
    const int ncu = md.ncu, nn = M.nn, nd = M.nd, nb = ncu * nn;
    const size_t N = (size_t)M.E * nb;
    std::vector<Dual> ud(N);
    for (size_t i = 0; i < N; ++i) ud[i] = Dual(u[i], v ? v[i] : 0.0);
    const size_t qsz = (size_t)ncu * nd * nn;
    std::vector<Dual> q(model_has_q(md) ? (size_t)M.E * qsz : 1);
    std::vector<Dual> RK(nb);
    for (int64_t s = 0; s < nsel; ++s) {
      long K = sel[s];
      if (model_has_q(md))
        for (long e : neighbourhood(M, K, 1)) compute_q(M, md, ud.data(), e, &q[(size_t)e * qsz]);
      element_residual(M, md, ud.data(), q.data(), K, RK.data());
      for (int i = 0; i < nb; ++i) {
        if (G) G[(size_t)s * nb + i] = RK[i].v;
        if (Jv) Jv[(size_t)s * nb + i] = RK[i].d;
      }
    }
  })
}

// consistent mass matrix applied element by element: Mu = M u
void ldgo_mass_apply(void* h, int ncu, const double* u, double* Mu) {
  OMesh& M = *(OMesh*)h;
  for (long K = 0; K < M.E; ++K) {
    std::vector<double> A = mass_matrix(M, K);
    for (int c = 0; c < ncu; ++c)
      for (int i = 0; i < M.nn; ++i) {
        double s = 0;
        for (int j = 0; j < M.nn; ++j) s += A[i * M.nn + j] * u[((size_t)K * ncu + c) * M.nn + j];
        Mu[((size_t)K * ncu + c) * M.nn + i] = s;
      }
  }
}

// Doolittle LU with partial pivoting, in place (row-major), piv[n]
int ldgo_lu_factor(int n, double* A, int* piv) {
  for (int k = 0; k < n; ++k) {
    int pr = k;
    double best = std::fabs(A[k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > best) { best = std::fabs(A[i * n + k]); pr = i; }
    piv[k] = pr;
    if (best == 0.0) { g_err = "singular block"; return -1; }
    if (pr != k)
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[pr * n + j]);
    for (int i = k + 1; i < n; ++i) {
      A[i * n + k] /= A[k * n + k];
      double l = A[i * n + k];
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
    }
  }
  return 0;
}

void ldgo_lu_solve(int n, const double* LU, const int* piv, double* b) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) std::swap(b[k], b[piv[k]]);
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int j = 0; j < i; ++j) s -= LU[i * n + j] * b[j];
    b[i] = s;
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= LU[i * n + j] * b[j];
    b[i] = s / LU[i * n + i];
  }
}

// O13: points of an independent Gauss-Legendre rule with m points per direction
// (for error norms) [E][m^nd][nd], and the relative L2 errors of u (component c)
// and of q against exact values sampled at those points.
void ldgo_error_points(void* h, int m, double* x) {
  OMesh& M = *(OMesh*)h;
  std::vector<double> xe, we;
  gauss_legendre(m, xe, we);
  int np = 1;
  for (int k = 0; k < M.nd; ++k) np *= m;
  int ie[3];
  for (long K = 0; K < M.E; ++K)
    for (int t = 0; t < np; ++t) {
      unflat(t, m, M.nd, ie);
      double xi[3], xx[3], J[9];
      for (int k = 0; k < M.nd; ++k) xi[k] = xe[ie[k]];
      map_point(M, K, xi, xx, J);
      for (int k = 0; k < M.nd; ++k) x[((size_t)K * np + t) * M.nd + k] = xx[k];
    }
}

// out[0] = ||u_h - u||, out[1] = ||u||, out[2] = ||q_h - q||, out[3] = ||q||  (component c)
void ldgo_l2_error(void* h, int m, int ncu, int c, const double* u, const double* q,
                   const double* uex, const double* qex, double* out) {
  OMesh& M = *(OMesh*)h;
  const int nd = M.nd, nn = M.nn;
  std::vector<double> xe, we;
  gauss_legendre(m, xe, we);
  int np = 1;
  for (int k = 0; k < nd; ++k) np *= m;
  int ie[3], in[3];
  double eu = 0, nu = 0, eq = 0, nq = 0;
  for (long K = 0; K < M.E; ++K)
    for (int t = 0; t < np; ++t) {
      unflat(t, m, nd, ie);
      double xi[3], xx[3], J[9], Ji[9];
      double w = 1.0;
      for (int k = 0; k < nd; ++k) { xi[k] = xe[ie[k]]; w *= we[ie[k]]; }
      map_point(M, K, xi, xx, J);
      double dj = det_and_inverse(nd, J, Ji);
      double uh = 0, qh[3] = {0, 0, 0};
      for (int i = 0; i < nn; ++i) {
        unflat(i, M.p + 1, nd, in);
        double phi = 1.0;
        for (int k = 0; k < nd; ++k) phi *= lagrange(M.xn, in[k], xi[k]);
        uh += u[((size_t)K * ncu + c) * nn + i] * phi;
        if (q)
          for (int k = 0; k < nd; ++k) qh[k] += q[(((size_t)K * ncu + c) * nd + k) * nn + i] * phi;
      }
      double ue = uex[(size_t)K * np + t];
      eu += w * dj * (uh - ue) * (uh - ue);
      nu += w * dj * ue * ue;
      if (q)
        for (int k = 0; k < nd; ++k) {
          double qe = qex[((size_t)K * np + t) * nd + k];
          eq += w * dj * (qh[k] - qe) * (qh[k] - qe);
          nq += w * dj * qe * qe;
        }
    }
  out[0] = std::sqrt(eu); out[1] = std::sqrt(nu); out[2] = std::sqrt(eq); out[3] = std::sqrt(nq);
}

// pointwise physical flux and numerical flux, for flux-level checks
int ldgo_point_flux(const ldgo_model_desc* d, int nd, const double* u, const double* q, const double* a, double* f) {
  GUARD({
    OModel md;
    md.kind = d->kind; md.ncu = d->ncu; md.naux = d->naux; md.nd = nd;
    md.mu.assign(d->mu, d->mu + d->nmu);
    phys_flux<double>(md, u, q, a, f);
  })
}
int ldgo_point_numflux(const ldgo_model_desc* d, int nd, const double* uL, const double* qL, const double* aL,
                       const double* uR, const double* qR, const double* aR, const double* n, double* Fh) {
  GUARD({
    OModel md;
    md.kind = d->kind; md.ncu = d->ncu; md.naux = d->naux; md.nd = nd;
    md.mu.assign(d->mu, d->mu + d->nmu);
    num_flux<double>(md, uL, qL, aL, uR, qR, aR, n, Fh);
  })
}

}  // extern "C"
