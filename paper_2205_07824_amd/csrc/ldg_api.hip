// C ABI: mesh set-up, model binding, residual and Jacobian-vector product.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "ldg_internal.hpp"
#include "ldg_physics.hpp"

namespace ldg {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

// ----------------------------------------------------------------------------
// Gauss-Legendre nodes/weights (Newton on P_m in long double) and the
// barycentric form of the Lagrange basis on them.
// ----------------------------------------------------------------------------
static void gl_rule(int m, std::vector<double>& x, std::vector<double>& w) {
  x.resize(m);
  w.resize(m);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < m; ++i) {
    long double z = cosl(pi * (m - i - 0.25L) / (m + 0.5L));  // ascending order
    long double pp = 0;
    for (int it = 0; it < 60; ++it) {
      long double p0 = 1, p1 = 0;
      for (int k = 0; k < m; ++k) {   // P_{k+1} = ((2k+1) z P_k - k P_{k-1}) / (k+1)
        long double p2 = p1;
        p1 = p0;
        p0 = ((2.0L * k + 1.0L) * z * p1 - k * p2) / (k + 1.0L);
      }
      pp = m * (z * p0 - p1) / (z * z - 1.0L);
      long double dz = p0 / pp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    if (m == 1) { z = 0; pp = 1; }
    x[i] = (double)z;
    w[i] = (double)(2.0L / ((1.0L - z * z) * pp * pp));
  }
}

static void make_basis(int p1, BasisTab& t, BasisTabF& tf) {
  std::memset(&t, 0, sizeof(t));
  std::vector<double> x, w;
  gl_rule(p1, x, w);
  long double lam[MAXP1];
  for (int a = 0; a < p1; ++a) {
    long double s = 1;
    for (int j = 0; j < p1; ++j)
      if (j != a) s *= ((long double)x[a] - x[j]);
    lam[a] = 1.0L / s;
  }
  for (int a = 0; a < p1; ++a) {
    t.x[a] = x[a];
    t.w[a] = w[a];
    long double diag = 0;
    for (int mm = 0; mm < p1; ++mm) {
      if (mm == a) continue;
      long double d = (lam[mm] / lam[a]) / ((long double)x[a] - x[mm]);
      t.D[a][mm] = (double)d;
      diag -= d;
    }
    t.D[a][a] = (double)diag;
  }
  for (int s = 0; s < 2; ++s) {
    long double tt = s ? 1.0L : -1.0L;
    long double den = 0;
    for (int j = 0; j < p1; ++j) den += lam[j] / (tt - x[j]);
    for (int mm = 0; mm < p1; ++mm) t.lf[s][mm] = (double)((lam[mm] / (tt - x[mm])) / den);
  }
  for (int a = 0; a < MAXP1; ++a) {
    tf.x[a] = (float)t.x[a];
    tf.w[a] = (float)t.w[a];
    for (int b = 0; b < MAXP1; ++b) tf.D[a][b] = (float)t.D[a][b];
    tf.lf[0][a] = (float)t.lf[0][a];
    tf.lf[1][a] = (float)t.lf[1][a];
  }
}

static void eval_map(const Mesh& m, int64_t K, const double* xi, double* x, double J[3][3]) {
  const int nd = m.nd;
  const double* c = &m.h_coef[(size_t)K * m.nv * nd];
  for (int i = 0; i < nd; ++i) {
    x[i] = 0;
    for (int j = 0; j < nd; ++j) J[i][j] = 0;
  }
  for (int mm = 0; mm < m.nv; ++mm) {
    double t = 1;
    for (int k = 0; k < nd; ++k)
      if ((mm >> k) & 1) t *= xi[k];
    for (int i = 0; i < nd; ++i) x[i] += c[mm * nd + i] * t;
    for (int j = 0; j < nd; ++j) {
      if (!((mm >> j) & 1)) continue;
      double tj = 1;
      for (int k = 0; k < nd; ++k)
        if (k != j && ((mm >> k) & 1)) tj *= xi[k];
      for (int i = 0; i < nd; ++i) J[i][j] += c[mm * nd + i] * tj;
    }
  }
}

struct KeyHash {
  size_t operator()(const std::vector<int64_t>& k) const {
    size_t h = 1469598103934665603ull;
    for (auto v : k) h = (h ^ (size_t)v) * 1099511628211ull;
    return h;
  }
};

}  // namespace ldg

using namespace ldg;


#define CHECK_ARG(cond, msg)           \
  do {                                 \
    if (!(cond)) {                     \
      set_error(msg);                  \
      return LDG_EINVAL;               \
    }                                  \
  } while (0)

extern "C" {

const char* ldg_last_error(void) { return g_err.c_str(); }

ldg_status ldg_mesh_create(int nd, int p, int nq1d, int64_t nvert, const double* vert, int64_t nelem,
                           const int64_t* elem_vert, const double* period, const int32_t* face_tag, ldg_mesh* out) {
  LDG_ENTER();
  CHECK_ARG(out && vert && elem_vert, "null argument");
  CHECK_ARG(nd == 2 || nd == 3, "nd must be 2 or 3");
  CHECK_ARG(p >= 1 && p + 1 <= MAXP1, "p must be in [1, 5]");
  CHECK_ARG(nq1d >= p + 1 && nq1d <= 16, "nq1d must be in [p+1, 16]");
  CHECK_ARG(nvert > 0 && nelem > 0 && nelem < (1ll << 31), "bad sizes");
  auto* m = new ldg_mesh_s();
  m->nd = nd; m->p = p; m->p1 = p + 1; m->nq1 = nq1d;
  m->nv = 1 << nd; m->nf = 2 * nd;
  m->nn = ipow(p + 1, nd); m->nfp = ipow(p + 1, nd - 1);
  m->nqv = ipow(nq1d, nd); m->nqf = ipow(nq1d, nd - 1);
  m->E = nelem;
  make_basis(p + 1, m->tab, m->tabf);
  gl_rule(nq1d, m->xq1, m->wq1);

  // element coordinates (periodic images unwrapped against the low corner) and
  // their multilinear monomial coefficients
  const int nv = m->nv;
  std::vector<double> X((size_t)nv * nd);
  m->h_coef.assign((size_t)nelem * nv * nd, 0.0);
  double scale = 0;
  for (int64_t i = 0; i < nvert * nd; ++i) scale = std::max(scale, std::fabs(vert[i]));
  scale = std::max(scale, 1.0);
  bool affine = true;
  for (int64_t K = 0; K < nelem; ++K) {
    for (int v = 0; v < nv; ++v) {
      int64_t vid = elem_vert[K * nv + v];
      if (vid < 0 || vid >= nvert) { delete m; set_error("vertex index out of range"); return LDG_EINVAL; }
      for (int k = 0; k < nd; ++k) {
        double c = vert[vid * nd + k];
        const double c0 = vert[elem_vert[K * nv] * nd + k];
        const double L = period ? period[k] : 0.0;
        if (L > 0) {
          while (c - c0 > 0.5 * L) c -= L;
          while (c0 - c >= 0.5 * L) c += L;
        }
        X[v * nd + k] = c;
      }
    }
    // C[mm] = (1/nv) sum_v (prod over the bits k of mm of +-1) X[v], as one
    // half-sum / half-difference butterfly per direction: a coefficient whose
    // corner values coincide (e.g. the xi_y term of x on an axis-aligned
    // element) comes out exactly zero, so axis-aligned faces get exactly
    // axis-aligned normals (a sequential signed sum left rounding residues of
    // ~1e-17, which gave random signs to normal velocities that are exactly
    // zero, e.g. w = 0 on z-faces, at the kink of |v.n|)
    double* C = &m->h_coef[(size_t)K * nv * nd];
    for (int t = 0; t < nv * nd; ++t) C[t] = X[t];
    for (int k = 0; k < nd; ++k)
      for (int v = 0; v < nv; ++v) {
        if ((v >> k) & 1) continue;
        const int w = v | (1 << k);
        for (int i = 0; i < nd; ++i) {
          const double lo = C[v * nd + i], hi = C[w * nd + i];
          C[v * nd + i] = 0.5 * (lo + hi);
          C[w * nd + i] = 0.5 * (hi - lo);
        }
      }
    for (int mm = 0; mm < nv; ++mm)
      if (__builtin_popcount(mm) >= 2)
        for (int i = 0; i < nd; ++i)
          if (std::fabs(C[mm * nd + i]) > 1e-13 * scale) affine = false;
    // positivity of det J at the corners and the centre
    for (int v = 0; v <= nv; ++v) {
      double xi[3] = {0, 0, 0}, x[3], J[3][3];
      if (v < nv)
        for (int k = 0; k < nd; ++k) xi[k] = ((v >> k) & 1) ? 1.0 : -1.0;
      eval_map(*m, K, xi, x, J);
      double det = nd == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                           : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      if (!(det > 0)) { delete m; set_error("element with non-positive Jacobian"); return LDG_EINVAL; }
    }
  }
  m->affine = affine;

  // faces keyed by sorted corner ids; every key must occur once (boundary) or twice
  const int nf = m->nf;
  m->h_nbr.assign((size_t)nelem * nf, INT32_MIN);
  std::unordered_map<std::vector<int64_t>, std::vector<std::pair<int64_t, int>>, KeyHash> faces;
  faces.reserve((size_t)nelem * nf);
  auto corners_of = [&](int64_t K, int F) {
    std::vector<int64_t> c;
    for (int v = 0; v < nv; ++v)
      if (((v >> (F >> 1)) & 1) == (F & 1)) c.push_back(elem_vert[K * nv + v]);
    return c;
  };
  for (int64_t K = 0; K < nelem; ++K)
    for (int F = 0; F < nf; ++F) {
      std::vector<int64_t> key = corners_of(K, F);
      std::sort(key.begin(), key.end());
      faces[key].emplace_back(K, F);
    }
  for (auto& kv : faces)
    if (kv.second.size() > 2) {
      delete m;
      set_error("face shared by more than two elements (or a periodic direction with fewer than 3 elements)");
      return LDG_EINVAL;
    }
  for (auto& kv : faces) {
    if (kv.second.size() != 2) continue;
    const int64_t K = kv.second[0].first, K2 = kv.second[1].first;
    const int F = kv.second[0].second, F2 = kv.second[1].second;
    if (K2 == K) { delete m; set_error("element adjacent to itself"); return LDG_EINVAL; }
    // required: opposite sides of the same reference direction, same tangential orientation
    if ((F2 >> 1) != (F >> 1) || (F2 & 1) == (F & 1) || corners_of(K, F) != corners_of(K2, F2)) {
      delete m;
      set_error("inconsistent face orientation between neighbouring elements");
      return LDG_EUNSUPPORTED;
    }
    m->h_nbr[(size_t)K * nf + F] = (int32_t)K2;
    m->h_nbr[(size_t)K2 * nf + F2] = (int32_t)K;
  }
  // boundary faces, element-major then local face
  m->nbf = 0;
  for (int64_t K = 0; K < nelem; ++K)
    for (int F = 0; F < nf; ++F)
      if (m->h_nbr[(size_t)K * nf + F] == INT32_MIN) {
        m->h_nbr[(size_t)K * nf + F] = -(int32_t)(1 + m->nbf);
        m->h_bface.push_back(K);
        m->h_bface.push_back(F);
        int32_t tg = face_tag ? face_tag[K * nf + F] : 0;
        m->h_btag.push_back(tg < 0 ? 0 : tg);
        ++m->nbf;
      }

  m->nbr_distinct = true;
  for (int64_t K = 0; K < nelem && m->nbr_distinct; ++K)
    for (int F = 0; F < nf; ++F) {
      const int32_t a = m->h_nbr[(size_t)K * nf + F];
      if (a < 0) continue;
      if (a == K) m->nbr_distinct = false;
      for (int F2 = F + 1; F2 < nf; ++F2)
        if (m->h_nbr[(size_t)K * nf + F2] == a) m->nbr_distinct = false;
    }
  // greedy distance-2 colouring of the element face graph
  m->h_color.assign(nelem, -1);
  m->ncolors = 0;
  std::vector<int64_t> ball;
  std::vector<char> used;
  for (int64_t K = 0; K < nelem; ++K) {
    ball.clear();
    for (int F = 0; F < nf; ++F) {
      int32_t n1 = m->h_nbr[(size_t)K * nf + F];
      if (n1 < 0) continue;
      ball.push_back(n1);
      for (int F2 = 0; F2 < nf; ++F2) {
        int32_t n2 = m->h_nbr[(size_t)n1 * nf + F2];
        if (n2 >= 0) ball.push_back(n2);
      }
    }
    used.assign(m->ncolors + 1, 0);
    for (int64_t e : ball)
      if (e != K && m->h_color[e] >= 0) used[m->h_color[e]] = 1;
    int c = 0;
    while (used[c]) ++c;
    m->h_color[K] = c;
    m->ncolors = std::max(m->ncolors, c + 1);
  }
  m->color_elems.assign(m->ncolors, {});
  for (int64_t K = 0; K < nelem; ++K) m->color_elems[m->h_color[K]].push_back((int32_t)K);
  std::vector<int32_t> clist;
  m->color_off.assign(m->ncolors + 1, 0);
  for (int c = 0; c < m->ncolors; ++c) {
    m->color_off[c] = (int64_t)clist.size();
    clist.insert(clist.end(), m->color_elems[c].begin(), m->color_elems[c].end());
  }
  m->color_off[m->ncolors] = (int64_t)clist.size();
  // per colour, the elements whose q tangent a JVP seeded on that colour needs
  // (the colour and its face neighbours)
  std::vector<int32_t> nlist;
  m->nbhd_off.assign(m->ncolors + 1, 0);
  {
    std::vector<int64_t> mark(nelem, -1);
    for (int c = 0; c < m->ncolors; ++c) {
      m->nbhd_off[c] = (int64_t)nlist.size();
      std::vector<int32_t> sc;
      for (int32_t K : m->color_elems[c]) {
        if (mark[K] != c) { mark[K] = c; sc.push_back(K); }
        for (int F = 0; F < nf; ++F) {
          const int32_t nb = m->h_nbr[(size_t)K * nf + F];
          if (nb >= 0 && mark[nb] != c) { mark[nb] = c; sc.push_back(nb); }
        }
      }
      std::sort(sc.begin(), sc.end());
      nlist.insert(nlist.end(), sc.begin(), sc.end());
    }
    m->nbhd_off[m->ncolors] = (int64_t)nlist.size();
  }

  // operator visit order.  3D: elements sorted by the Morton code of their
  // centroid (the constant monomial coefficient), so that the work-groups in
  // flight on one XCD touch face neighbours that are also in flight and share
  // its L2 (measured 15% faster on the 64^3 Navier-Stokes tangent).  2D: the
  // input order, whose neighbour rows already fit in L2 (Morton measured a few
  // per cent slower there).
  m->h_order.resize(nelem);
  for (int64_t K = 0; K < nelem; ++K) m->h_order[K] = (int32_t)K;
  if (nd == 3) {
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int k = 0; k < nd; ++k) { lo[k] = 1e300; hi[k] = -1e300; }
    for (int64_t K = 0; K < nelem; ++K)
      for (int k = 0; k < nd; ++k) {
        const double c = m->h_coef[(size_t)K * nv * nd + k];
        lo[k] = std::min(lo[k], c);
        hi[k] = std::max(hi[k], c);
      }
    const int bits = 10;
    std::vector<uint64_t> code((size_t)nelem, 0);
    for (int64_t K = 0; K < nelem; ++K) {
      uint64_t cell[3] = {0, 0, 0};
      for (int k = 0; k < nd; ++k) {
        const double ext = hi[k] - lo[k];
        double t = ext > 0 ? (m->h_coef[(size_t)K * nv * nd + k] - lo[k]) / ext : 0.0;
        t = std::min(std::max(t, 0.0), 1.0);
        cell[k] = std::min<uint64_t>((uint64_t)(t * double(1u << bits)), (1u << bits) - 1);
      }
      uint64_t z = 0;
      for (int b = bits - 1; b >= 0; --b)
        for (int k = nd - 1; k >= 0; --k) z = (z << 1) | ((cell[k] >> b) & 1u);
      code[K] = z;
    }
    std::stable_sort(m->h_order.begin(), m->h_order.end(), [&](int32_t a, int32_t b) { return code[a] < code[b]; });
  }

  // upload
  hipError_t e = hipSuccess;
  e = hipMalloc((void**)&m->d_coef, m->h_coef.size() * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(m->d_coef, m->h_coef.data(), m->h_coef.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_nbr, m->h_nbr.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemcpy(m->d_nbr, m->h_nbr.data(), m->h_nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_btag, std::max<size_t>(1, m->h_btag.size()) * sizeof(int32_t));
  if (e == hipSuccess && !m->h_btag.empty())
    e = hipMemcpy(m->d_btag, m->h_btag.data(), m->h_btag.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_color_list, clist.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemcpy(m->d_color_list, clist.data(), clist.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_color_nbhd, std::max<size_t>(1, nlist.size()) * sizeof(int32_t));
  if (e == hipSuccess && !nlist.empty())
    e = hipMemcpy(m->d_color_nbhd, nlist.data(), nlist.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc((void**)&m->d_order, m->h_order.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemcpy(m->d_order, m->h_order.data(), m->h_order.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    set_error(std::string("mesh upload: ") + hipGetErrorString(e));
    hipFree(m->d_coef); hipFree(m->d_nbr); hipFree(m->d_btag); hipFree(m->d_color_list); hipFree(m->d_color_nbhd);
    hipFree(m->d_order);
    delete m;
    return e == hipErrorOutOfMemory ? LDG_ENOMEM : LDG_EDEVICE;
  }
  *out = m;
  return LDG_OK;
}

ldg_status ldg_mesh_info(ldg_mesh m, int64_t* info) {
  LDG_ENTER();
  CHECK_ARG(m && info, "null argument");
  info[0] = m->E; info[1] = m->nn; info[2] = m->nqv; info[3] = m->nqf; info[4] = m->nbf;
  info[5] = m->ncolors; info[6] = m->affine ? 1 : 0; info[7] = m->nd;
  return LDG_OK;
}

ldg_status ldg_mesh_points(ldg_mesh m, double* xnode, double* xquad, double* xbface, int64_t* bface) {
  LDG_ENTER();
  CHECK_ARG(m, "null mesh");
  const int nd = m->nd;
  double x[3], J[3][3], xi[3];
  for (int64_t K = 0; K < m->E; ++K) {
    if (xnode)
      for (int i = 0; i < m->nn; ++i) {
        int t = i;
        for (int k = 0; k < nd; ++k) { xi[k] = m->tab.x[t % m->p1]; t /= m->p1; }
        eval_map(*m, K, xi, x, J);
        for (int k = 0; k < nd; ++k) xnode[((size_t)K * m->nn + i) * nd + k] = x[k];
      }
    if (xquad)
      for (int i = 0; i < m->nqv; ++i) {
        int t = i;
        for (int k = 0; k < nd; ++k) { xi[k] = m->xq1[t % m->nq1]; t /= m->nq1; }
        eval_map(*m, K, xi, x, J);
        for (int k = 0; k < nd; ++k) xquad[((size_t)K * m->nqv + i) * nd + k] = x[k];
      }
  }
  for (int64_t b = 0; b < m->nbf; ++b) {
    const int64_t K = m->h_bface[2 * b];
    const int F = (int)m->h_bface[2 * b + 1];
    if (bface) { bface[2 * b] = K; bface[2 * b + 1] = F; }
    if (!xbface) continue;
    const int dir = F >> 1, side = F & 1;
    for (int f = 0; f < m->nqf; ++f) {
      int t = f;
      for (int k = 0; k < nd; ++k) {
        if (k == dir) { xi[k] = side ? 1.0 : -1.0; continue; }
        xi[k] = m->xq1[t % m->nq1];
        t /= m->nq1;
      }
      eval_map(*m, K, xi, x, J);
      for (int k = 0; k < nd; ++k) xbface[((size_t)b * m->nqf + f) * nd + k] = x[k];
    }
  }
  return LDG_OK;
}

ldg_status ldg_mesh_destroy(ldg_mesh m) {
  LDG_ENTER();
  if (!m) return LDG_OK;
  hipFree(m->d_coef); hipFree(m->d_nbr); hipFree(m->d_btag); hipFree(m->d_color_list); hipFree(m->d_color_nbhd);
    hipFree(m->d_order);
  delete m;
  return LDG_OK;
}

static ldg_status model_create(ldg_mesh m, const ldg_model_desc* d, const char* user_source, int has_q, void* stream,
                               ldg_model* out) {
  CHECK_ARG(m && d && out, "null argument");
  {
    // operator kernels are compiled for quads with p <= 4 and hexes with p <= 3
    const ldg::Mesh& mm = *m;
    if ((mm.nd == 2 && mm.p1 > 5) || (mm.nd == 3 && mm.p1 > 4)) {
      set_error("no operator kernels for this order: quads take p <= 4, hexes p <= 3");
      return LDG_EUNSUPPORTED;
    }
  }
  const bool user = user_source != nullptr;
  if (user) {
    CHECK_ARG(d->kind == LDG_MODEL_USER, "a physics source needs kind LDG_MODEL_USER");
    CHECK_ARG(d->ncu >= 1 && d->ncu <= 8, "ncu must be in [1, 8]");
  } else {
    CHECK_ARG(d->kind >= 0 && d->kind <= 3, "unknown model kind (LDG_MODEL_USER needs ldg_model_create_user)");
    const int want_ncu = d->kind <= 1 ? 1 : m->nd + 2;
    CHECK_ARG(d->ncu == want_ncu, "ncu inconsistent with the model");
  }
  CHECK_ARG(d->nmu >= 0 && d->nmu <= MAXMU && (d->nmu == 0 || d->mu), "bad mu");
  CHECK_ARG(d->nbc >= 1 && d->nbc <= MAXTAG && d->bc_kind, "need 1..8 boundary kinds");
  CHECK_ARG(d->naux >= 0 && (d->naux == 0 || d->aux), "bad aux");
  if (d->kind == LDG_MODEL_CONVDIFF) CHECK_ARG(d->naux == 1 + m->nd, "convection-diffusion needs aux = [kappa, b]");
  if (d->kind == LDG_MODEL_POISSON) CHECK_ARG(d->naux <= 1, "Poisson takes at most one aux field");
  if (d->kind == LDG_MODEL_EULER || d->kind == LDG_MODEL_NS) CHECK_ARG(d->naux == 0, "Euler / NS take no aux fields");
  for (int i = 0; i < d->nbc; ++i) CHECK_ARG(d->bc_kind[i] >= 0 && d->bc_kind[i] <= 2, "bad bc kind");
  if (m->nq1 != m->p1) {
    if (!(d->kind == LDG_MODEL_POISSON && d->naux == 0 && m->affine)) {
      set_error("nq1d > p+1 is supported only for Poisson with constant kappa on affine meshes");
      return LDG_EUNSUPPORTED;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  auto* md = new ldg_model_s();
  md->mesh = m;
  md->kind = d->kind; md->ncu = d->ncu; md->nmu = d->nmu; md->naux = d->naux;
  for (int i = 0; i < MAXMU; ++i) md->mu[i] = i < d->nmu ? d->mu[i] : 0.0;
  // defaults for missing parameters
  if (user) {
    // no defaults: the physics source reads mu as given
  } else if (d->kind <= 1) {
    if (d->nmu < 1) md->mu[0] = 1.0;
    if (d->nmu < 2) md->mu[1] = 1.0;
  } else {
    if (d->nmu < 1) md->mu[0] = 1.4;
    if (d->kind == 3) {
      if (d->nmu < 2) md->mu[1] = 1.0;
      if (d->nmu < 3) md->mu[2] = 0.72;
      if (d->nmu < 4) md->mu[3] = 1.0;
    }
  }
  md->nbc = d->nbc;
  for (int i = 0; i < MAXTAG; ++i) md->bc_kind[i] = i < d->nbc ? d->bc_kind[i] : d->bc_kind[d->nbc - 1];
  md->aux = d->aux; md->src = d->src; md->bdata = d->bdata;
  md->linear = d->kind <= 1;
  md->hasq = user ? has_q != 0 : d->kind != LDG_MODEL_EULER;
  const size_t N = md->N();
  const size_t NQ = N * m->nd;
  hipError_t e = hipSuccess;
  e = hipMalloc((void**)&md->d_q, NQ * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&md->d_q32, NQ * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&md->d_qres, NQ * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&md->d_dq, NQ * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&md->d_tmp, N * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&md->d_tmp2, N * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&md->d_red, 4096 * sizeof(double));
  if (e == hipSuccess && md->linear) {
    e = hipMalloc((void**)&md->d_qg, NQ * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void**)&md->d_dterm, N * sizeof(double));
  }
  if (e != hipSuccess) {
    set_error(std::string("model allocation: ") + hipGetErrorString(e));
    ldg_model_destroy(md);
    return LDG_ENOMEM;
  }
  if (md->linear) {
    ldg_status st = op_data_terms(*md, s);
    if (st == LDG_OK) st = mfma_prepare(*md);
    if (st != LDG_OK) { ldg_model_destroy(md); return st; }
  } else {
    md->d_srcn = const_cast<double*>(d->src);   // collocated: quadrature points are the nodes
  }
  if (user) {
    ldg_status st = jit_build(*md, user_source);
    if (st != LDG_OK) { ldg_model_destroy(md); return st; }
  }
  *out = md;
  return LDG_OK;
}

ldg_status ldg_model_create(ldg_mesh m, const ldg_model_desc* d, void* stream, ldg_model* out) {
  LDG_ENTER();
  return model_create(m, d, nullptr, 1, stream, out);
}

ldg_status ldg_model_create_user(ldg_mesh m, const ldg_model_desc* d, const char* physics_source, int has_q,
                                 void* stream, ldg_model* out) {
  LDG_ENTER();
  CHECK_ARG(physics_source, "null physics source");
  return model_create(m, d, physics_source, has_q, stream, out);
}

ldg_status ldg_user_physics_check(const char* physics_source, int nd, int p, int ncu, int has_q) {
  LDG_ENTER();
  CHECK_ARG(physics_source, "null physics source");
  CHECK_ARG((nd == 2 && p >= 1 && p <= 4) || (nd == 3 && p >= 1 && p <= 3),
            "operator kernels exist for quads with p <= 4 and hexes with p <= 3");
  CHECK_ARG(ncu >= 1 && ncu <= 8, "ncu must be in [1, 8]");
  return jit_check(physics_source, nd, p + 1, ncu, has_q != 0);
}

ldg_status ldg_ode_size(ldg_model md, int* nw) {
  LDG_ENTER();
  CHECK_ARG(md && nw, "null argument");
  *nw = jit_ode_size(*md);
  return LDG_OK;
}

ldg_status ldg_ode_stage(ldg_model md, const ldg_time* t, double alpha, double beta, const double* u, double* w,
                         void* stream) {
  LDG_ENTER();
  CHECK_ARG(md && t && u && w, "null argument");
  CHECK_ARG((const double*)w != u, "w must not alias u");
  CHECK_ARG(alpha * t->a0 + beta != 0.0, "alpha a0 + beta must not vanish");
  if (jit_ode_size(*md) == 0) {
    set_error("the model defines no ODE (a physics source with LdgUser::NW and ode_source)");
    return LDG_EUNSUPPORTED;
  }
  return jit_ode(*md, make_time(t, true), alpha, beta, u, w, (hipStream_t)stream);
}

ldg_status ldg_model_destroy(ldg_model md) {
  LDG_ENTER();
  if (!md) return LDG_OK;
  mfma_release(*md);
  jit_release(*md);
  hipFree(md->d_q); hipFree(md->d_tr); hipFree(md->d_trt); hipFree(md->d_probe); hipFree(md->d_tr32); hipFree(md->d_q32); hipFree(md->d_qres); hipFree(md->d_dq); hipFree(md->d_tmp); hipFree(md->d_tmp2); hipFree(md->d_red);
  hipFree(md->d_qg); hipFree(md->d_dterm);
  delete md;
  return LDG_OK;
}

}  // extern "C"

namespace ldg {

TimeDev make_time(const ldg_time* t, bool with_rhs) {
  TimeDev d{0.0, 0.0, 0.0, nullptr, nullptr};
  if (!t) return d;
  d.a0 = t->a0;
  if (with_rhs) {
    d.r1 = t->r1; d.c1 = t->c1;
    d.r2 = t->r2; d.c2 = t->c2;
  }
  return d;
}

__global__ void k_f32_to_f64(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

ldg_status residual_impl(Model& md, const ldg_time* t, const double* u, double* G, double* q_out, bool fp32,
                         hipStream_t s) {
  void* qbuf = (!fp32 && q_out) ? (void*)q_out : (void*)md.d_qres;
  ldg_status st = op_grad(md, u, qbuf, fp32, true, s);
  if (st != LDG_OK) return st;
  st = op_resid(md, make_time(t, true), u, qbuf, G, fp32, true, s);
  if (st != LDG_OK) return st;
  if (q_out && qbuf != q_out && md.hasq) {
    const int64_t n = (int64_t)md.N() * md.mesh->nd;
    hipLaunchKernelGGL(k_f32_to_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, (const float*)qbuf, q_out);
    LDG_TRY(hipGetLastError());
  }
  return LDG_OK;
}

// J(u) v with u, v in FP32 storage (FP32 arithmetic); for nonlinear models q
// comes from md.d_q32 (prepared = true) or is formed here from the FP32 state.
ldg_status jvp_state32(Model& md, const ldg_time* t, const float* u, const float* v, double* Jv,
                              bool prepared, hipStream_t s) {
  const TimeDev td = make_time(t, false);
  ldg_status st = op_grad(md, v, md.d_dq, PM_FP32_STATE, false, s);
  if (st != LDG_OK) return st;
  if (md.linear) return op_resid(md, td, v, md.d_dq, Jv, PM_FP32_STATE, false, s);
  if (!u) {
    set_error("nonlinear model needs u");
    return LDG_EINVAL;
  }
  if (!prepared && md.hasq) {
    // the cache now holds q of an FP32 state, which no FP64 pointer names
    st = form_q_cache32(md, u, PM_FP32_STATE, s);
    if (st != LDG_OK) return st;
  }
  return op_jvp_nonlinear(md, td, u, md.d_q32, v, md.d_dq, Jv, PM_FP32_STATE, s);
}

// J(u) v; for nonlinear models q(u) must already be in md.d_q (prepared = true)
// or is computed here.
ldg_status jvp_impl(Model& md, const ldg_time* t, const double* u, const double* v, double* Jv, ldg_precision prec,
                    bool prepared, hipStream_t s) {
  if (prec == LDG_JVP_FD) {
    // one-sided difference, eps = sqrt(macheps) (1 + ||u||) / ||v|| (Knoll & Keyes 2004)
    const int64_t n = (int64_t)md.N();
    double nu = 0.0, nv = 0.0;
    ldg_status st;
    if (u) { st = vec_norm2(n, u, md.d_red, &nu, s); if (st != LDG_OK) return st; }
    st = vec_norm2(n, v, md.d_red, &nv, s);
    if (st != LDG_OK) return st;
    if (nv == 0.0) return vec_fill(n, 0.0, Jv, s);
    const double eps = 1.4901161193847656e-08 * (1.0 + std::sqrt(nu)) / std::sqrt(nv);
    if (u) LDG_TRY(hipMemcpyAsync(md.d_tmp, u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    else if ((st = vec_fill(n, 0.0, md.d_tmp, s)) != LDG_OK) return st;
    if ((st = residual_impl(md, t, md.d_tmp, Jv, nullptr, false, s)) != LDG_OK) return st;
    if ((st = vec_axpby(n, eps, v, 1.0, md.d_tmp, s)) != LDG_OK) return st;
    if ((st = residual_impl(md, t, md.d_tmp, md.d_tmp2, nullptr, false, s)) != LDG_OK) return st;
    return vec_axpby(n, 1.0 / eps, md.d_tmp2, -1.0 / eps, Jv, s);
  }
  if (prec == LDG_BF16_MFMA || prec == LDG_FP16_MFMA) {
    if (!md.linear) {
      set_error("MFMA JVP is implemented for the linear models");
      return LDG_EUNSUPPORTED;
    }
    return op_mfma_jvp(md, make_time(t, false), v, Jv, prec == LDG_FP16_MFMA, s);
  }
  if (prec != LDG_FP64 && prec != LDG_FP32) {
    set_error("unknown precision");
    return LDG_EINVAL;
  }
  const bool fp32 = prec == LDG_FP32;
  const TimeDev td = make_time(t, false);
  if (md.linear) {
    ldg_status st = op_grad(md, v, md.d_dq, fp32, false, s);
    if (st != LDG_OK) return st;
    return op_resid(md, td, v, md.d_dq, Jv, fp32, false, s);
  }
  if (!u) {
    set_error("nonlinear model needs u");
    return LDG_EINVAL;
  }
  ldg_status st;
  void* qc = fp32 ? (void*)md.d_q32 : (void*)md.d_q;
  if (!prepared && md.hasq) {
    if (fp32) {
      if ((st = form_q_cache32(md, u, PM_FP32, s)) != LDG_OK) return st;
    } else if ((st = form_q_cache64(md, u, s)) != LDG_OK) {
      return st;
    }
  }
  if (md.hasq) {
    st = op_grad(md, v, md.d_dq, fp32, false, s);
    if (st != LDG_OK) return st;
  }
  return op_jvp_nonlinear(md, td, u, qc, v, md.d_dq, Jv, fp32, s);
}

}  // namespace ldg

extern "C" {

ldg_status ldg_residual(ldg_model md, const ldg_time* t, const double* u, double* G, double* q_out, ldg_precision prec,
                        void* stream) {
  LDG_ENTER();
  CHECK_ARG(md && u && G, "null argument");
  CHECK_ARG(prec == LDG_FP64 || prec == LDG_FP32, "residual precision must be FP64 or FP32");
  return residual_impl(*md, t, u, G, q_out, prec == LDG_FP32, (hipStream_t)stream);
}

ldg_status ldg_jvp(ldg_model md, const ldg_time* t, const double* u, const double* v, double* Jv, ldg_precision prec,
                   void* stream) {
  LDG_ENTER();
  CHECK_ARG(md && v && Jv, "null argument");
  CHECK_ARG(Jv != v && Jv != u, "Jv must not alias u or v");
  return jvp_impl(*md, t, u, v, Jv, prec, false, (hipStream_t)stream);
}

ldg_status ldg_jvp_state32(ldg_model md, const ldg_time* t, const float* u, const float* v, double* Jv,
                           void* stream) {
  LDG_ENTER();
  CHECK_ARG(md && v && Jv, "null argument");
  CHECK_ARG((const void*)Jv != (const void*)v && (const void*)Jv != (const void*)u, "Jv must not alias u or v");
  return jvp_state32(*md, t, u, v, Jv, false, (hipStream_t)stream);
}

ldg_status ldg_jvp_prepare(ldg_model md, const double* u, ldg_precision prec, void* stream) {
  LDG_ENTER();
  CHECK_ARG(md && u, "null argument");
  CHECK_ARG(prec == LDG_FP64 || prec == LDG_FP32, "ldg_jvp_prepare: precision must be FP64 or FP32");
  if (md->linear || !md->hasq) return LDG_OK;
  const bool fp32 = prec == LDG_FP32;
  if (!fp32) return form_q_cache64(*md, u, (hipStream_t)stream);
  return form_q_cache32(*md, u, PM_FP32, (hipStream_t)stream);
}

ldg_status ldg_jvp_prepared(ldg_model md, const ldg_time* t, const double* u, const double* v, double* Jv,
                            ldg_precision prec, void* stream) {
  LDG_ENTER();
  CHECK_ARG(md && v && Jv, "null argument");
  CHECK_ARG(Jv != v && Jv != u, "Jv must not alias u or v");
  if (prec != LDG_FP64 && prec != LDG_FP32) return jvp_impl(*md, t, u, v, Jv, prec, false, (hipStream_t)stream);
  if (!md->linear && md->hasq) {
    CHECK_ARG(u != nullptr, "nonlinear model needs u");
    if (md->q_of[prec == LDG_FP32 ? 1 : 0] != u) {
      set_error("ldg_jvp_prepared: q of this u is not cached in this precision (call ldg_jvp_prepare first; "
                "solver and preconditioner calls on the model replace the cache)");
      return LDG_EINVAL;
    }
  }
  return jvp_impl(*md, t, u, v, Jv, prec, true, (hipStream_t)stream);
}

ldg_status ldg_axpby(int64_t n, double a, const double* x, double b, double* y, void* stream) {
  LDG_ENTER();
  CHECK_ARG(n >= 0 && x && y, "bad arguments");
  return vec_axpby(n, a, x, b, y, (hipStream_t)stream);
}

ldg_status ldg_norm2(int64_t n, const double* x, double* out, void* stream) {
  LDG_ENTER();
  CHECK_ARG(n >= 0 && x && out, "bad arguments");
  double* part = nullptr;
  LDG_TRY(hipMalloc((void**)&part, 4096 * sizeof(double)));   // reduction partials + result slot
  ldg_status st = vec_norm2(n, x, part, out, (hipStream_t)stream);
  hipFree(part);
  return st;
}

}  // extern "C"
