// FP64 Krylov machinery for the matrix-free Newton-GMRES solver (Section 3.3):
// vector kernels, the block-wise multi-dot / update pair of classical
// Gram-Schmidt with one re-orthogonalization pass (CGS2), Givens rotations on
// the device, restarted flexible GMRES, and Newton's method.
#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cstring>
#include <cmath>

#include "ldg_internal.hpp"

namespace ldg {

constexpr int RED_BLOCKS = 1024;   // partial-sum slots per reduction
constexpr int VB = 256;            // threads per block of the vector kernels

// ---------------------------------------------------------------- vectors ---
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}
__global__ void k_zero_int(int* p) { if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0; }
ldg_status zero_int(int* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, s, p);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}
__global__ void k_fill(int64_t n, double a, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = a;
}
__global__ void k_scale_dev(int64_t n, const double* __restrict__ sc, const double* __restrict__ x,
                            double* __restrict__ y) {
  const double a = *sc;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

// y -= a[0] x (a on the device)
__global__ void k_axmy_dev(int64_t n, const double* __restrict__ a, const double* __restrict__ x,
                           double* __restrict__ y) {
  const double c = *a;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] -= c * x[i];
}

__device__ inline double block_sum(double v, double* sh) {
  // wave64 shuffle reduction, then across waves through LDS
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

__global__ void k_dot_partial(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                              double* __restrict__ part) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_partials(int nparts, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *out = s;
}

static int grid_for(int64_t n) {
  int64_t g = (n + VB - 1) / VB;
  if (g > RED_BLOCKS) g = RED_BLOCKS;
  if (g < 1) g = 1;
  return (int)g;
}

ldg_status vec_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (n == 0) return LDG_OK;
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(VB), 0, s, n, a, x, b, y);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}
ldg_status vec_fill(int64_t n, double a, double* y, hipStream_t s) {
  if (n == 0) return LDG_OK;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(VB), 0, s, n, a, y);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}
// sum(x^2) to the host; part needs >= RED_BLOCKS + 1 doubles
ldg_status vec_norm2(int64_t n, const double* x, double* part, double* host_out, hipStream_t s) {
  const int g = grid_for(n);
  hipLaunchKernelGGL(k_dot_partial, dim3(g), dim3(VB), 0, s, n, x, x, part);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(VB), 0, s, g, part, part + RED_BLOCKS);
  LDG_TRY(hipGetLastError());
  LDG_TRY(hipMemcpyAsync(host_out, part + RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, s));
  LDG_TRY(hipStreamSynchronize(s));
  return LDG_OK;
}

// ------------------------------------------------------- Gram-Schmidt sweeps ---
// Classical Gram-Schmidt with one re-orthogonalization (CGS2), as three streaming
// sweeps over the basis V per Arnoldi step, each reading every basis vector once:
//   A  h1 = V^T w, ||w||^2                       (k_cgs_dots)
//   B  w -= V h1 ; h2 = V^T w                    (k_cgs_update_dots, nv <= 32)
//   C  w -= V h2 ; ||w||^2                       (k_cgs_update)
// Each work-group owns a contiguous chunk of the vectors; a thread keeps up to G
// basis values and G dot accumulators in registers, so all loads of one element
// index are independent.  Block partials go to part[i * nblk + b] and are reduced
// by k_reduce_rows (deterministic, no atomics).
constexpr int MAXM = 512;   // largest restart length (Krylov basis size)

__device__ inline void chunk_of(int64_t n, int64_t* lo, int64_t* hi) {
  const int nblk = gridDim.x;
  const int64_t chunk = ((n + nblk - 1) / nblk + VB - 1) / VB * VB;
  *lo = (int64_t)blockIdx.x * chunk;
  *hi = *lo + chunk < n ? *lo + chunk : n;
}

// block reduction of nr <= G values per thread; threads 0..nr-1 return the sums
template <int G>
__device__ inline double block_sum_many(const double (&s)[G], int nr, double (*sh)[G]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < G; ++r) {
    if (r < nr) {
      double v = s[r];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) sh[wid][r] = v;
    }
  }
  __syncthreads();
  double t = 0.0;
  if ((int)threadIdx.x < nr)
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += sh[w][threadIdx.x];
  __syncthreads();
  return t;
}

// A: part rows i < nv: V_i . w; row nv: w . w
template <int G>
__global__ void __launch_bounds__(VB) k_cgs_dots(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double sh[VB / 64][G + 1];
  int64_t lo, hi;
  chunk_of(n, &lo, &hi);
  const int nblk = gridDim.x;
  for (int i0 = 0; i0 < nv; i0 += G) {
    const int ni = nv - i0 < G ? nv - i0 : G;
    double s[G + 1];
#pragma unroll
    for (int r = 0; r <= G; ++r) s[r] = 0.0;
    for (int64_t t = lo + threadIdx.x; t < hi; t += VB) {
      const double wt = w[t];
      double v[G];
#pragma unroll
      for (int r = 0; r < G; ++r) v[r] = (r < ni) ? V[(int64_t)(i0 + r) * ldv + t] : 0.0;
#pragma unroll
      for (int r = 0; r < G; ++r) s[r] += v[r] * wt;
      s[G] += wt * wt;
    }
    // the norm rides in slot ni of the first group
    const int nr = (i0 == 0) ? ni + 1 : ni;
    if (i0 == 0) {
#pragma unroll
      for (int r = 0; r < G; ++r)
        if (r == ni) s[r] = s[G];
    }
    const double tot = block_sum_many<G + 1>(s, nr, sh);
    if ((int)threadIdx.x < nr) {
      const int row = (i0 == 0 && (int)threadIdx.x == ni) ? nv : i0 + (int)threadIdx.x;
      part[(int64_t)row * nblk + blockIdx.x] = tot;
    }
  }
}

// B: w -= V h ; part rows i < nv: V_i . w  (nv <= G)
template <int G>
__global__ void __launch_bounds__(VB) k_cgs_update_dots(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                                        const double* __restrict__ h, double* __restrict__ w,
                                                        double* __restrict__ part) {
  __shared__ double sh[VB / 64][G];
  __shared__ double hs[G];
  for (int i = threadIdx.x; i < G; i += blockDim.x) hs[i] = i < nv ? h[i] : 0.0;
  __syncthreads();
  int64_t lo, hi;
  chunk_of(n, &lo, &hi);
  double s[G];
#pragma unroll
  for (int r = 0; r < G; ++r) s[r] = 0.0;
  for (int64_t t = lo + threadIdx.x; t < hi; t += VB) {
    double v[G];
#pragma unroll
    for (int r = 0; r < G; ++r) v[r] = (r < nv) ? V[(int64_t)r * ldv + t] : 0.0;
    double acc = w[t];
#pragma unroll
    for (int r = 0; r < G; ++r) acc -= hs[r] * v[r];
    w[t] = acc;
#pragma unroll
    for (int r = 0; r < G; ++r) s[r] += v[r] * acc;
  }
  const double tot = block_sum_many<G>(s, nv, sh);
  if ((int)threadIdx.x < nv) part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = tot;
}

// C: w -= V h (any nv, groups of G) ; npart (nullable) = block partials of w . w
template <int G>
__global__ void __launch_bounds__(VB) k_cgs_update(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ h, double* __restrict__ w,
                                                   double* __restrict__ npart) {
  __shared__ double sh[VB / 64][1];
  __shared__ double hs[MAXM + 1];
  for (int i = threadIdx.x; i < nv; i += blockDim.x) hs[i] = h[i];
  __syncthreads();
  int64_t lo, hi;
  chunk_of(n, &lo, &hi);
  double ss[1] = {0.0};
  for (int64_t t = lo + threadIdx.x; t < hi; t += VB) {
    double acc = w[t];
    for (int i0 = 0; i0 < nv; i0 += G) {
      double v[G];
#pragma unroll
      for (int r = 0; r < G; ++r) v[r] = (i0 + r < nv) ? V[(int64_t)(i0 + r) * ldv + t] : 0.0;
#pragma unroll
      for (int r = 0; r < G; ++r)
        if (i0 + r < nv) acc -= hs[i0 + r] * v[r];
    }
    w[t] = acc;
    ss[0] += acc * acc;
  }
  const double tot = block_sum_many<1>(ss, 1, sh);
  if (threadIdx.x == 0 && npart) npart[blockIdx.x] = tot;
}

// reduce the partials of nv dot products into h[0..nv) (one block per dot)
__global__ void k_reduce_rows(int nv, int nblk, const double* __restrict__ part, double* __restrict__ h) {
  __shared__ double sh[16];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += part[(int64_t)i * nblk + b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0 && i < nv) h[i] = s;
}

// x += sum_i y_i Z_i
// x += Z y (Z in FP64, or FP32 for the FP32-state solver)
template <class ZT>
__global__ void k_combine(int64_t n, int k, const ZT* __restrict__ Z, int64_t ldz, const double* __restrict__ y,
                          double* __restrict__ x) {
  __shared__ double ys[MAXM];
  for (int i = threadIdx.x; i < k; i += blockDim.x) ys[i] = y[i];
  __syncthreads();
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double acc = x[t];
    for (int i = 0; i < k; ++i) acc += ys[i] * (double)Z[(int64_t)i * ldz + t];
    x[t] = acc;
  }
}

// Arnoldi bookkeeping on the device, FP64, one block:
//  column j of H = h1 + h2 (two Gram-Schmidt passes), h_{j+1,j} = ||w||,
//  apply the previous rotations, build rotation j (hypot), update g,
//  write 1/h_{j+1,j} for the normalization and |g_{j+1}|, breakdown flag.
struct ArnoldiState {
  double H[(MAXM + 1) * MAXM];   // column-major, ld = MAXM + 1
  double cs[MAXM], sn[MAXM], g[MAXM + 1], y[MAXM];
  double inv_hnext;
  double resid;                  // |g_{j+1}|
  int breakdown;                 // directly after resid: one 16-byte copy reads both
  int pad_;
  double wnorm0;                 // ||w|| before orthogonalization
  double sigma;                  // delayed variant: the factor the pending vector U was divided by
};
static_assert(offsetof(ArnoldiState, breakdown) == offsetof(ArnoldiState, resid) + sizeof(double),
              "resid and breakdown are copied to the host together");

// h1[j + 1] holds ||w||^2 before the orthogonalization.  The column and the
// previous rotations are staged in LDS, so that the sequential rotation chain
// of thread 0 reads no global memory.
__global__ void k_givens(ArnoldiState* st, int j, int nblk, const double* __restrict__ h1, const double* __restrict__ h2,
                         const double* __restrict__ npart) {
  __shared__ double sh[16];
  __shared__ double colL[MAXM + 1], csL[MAXM], snL[MAXM];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += npart[b];
  s = block_sum(s, sh);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) colL[i] = h1[i] + h2[i];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    csL[i] = st->cs[i];
    snL[i] = st->sn[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->wnorm0 = sqrt(h1[j + 1]);
    const double hn = sqrt(s);
    colL[j + 1] = hn;
    st->breakdown = (hn <= 1e-14 * st->wnorm0) ? 1 : 0;
    st->inv_hnext = hn > 0 ? 1.0 / hn : 0.0;
    for (int i = 0; i < j; ++i) {
      const double t = csL[i] * colL[i] + snL[i] * colL[i + 1];
      colL[i + 1] = -snL[i] * colL[i] + csL[i] * colL[i + 1];
      colL[i] = t;
    }
    const double d = hypot(colL[j], colL[j + 1]);
    st->cs[j] = d > 0 ? colL[j] / d : 1.0;
    st->sn[j] = d > 0 ? colL[j + 1] / d : 0.0;
    colL[j] = d;
    colL[j + 1] = 0.0;
    st->g[j + 1] = -st->sn[j] * st->g[j];
    st->g[j] = st->cs[j] * st->g[j];
    st->resid = fabs(st->g[j + 1]);
  }
  __syncthreads();
  double* col = st->H + (int64_t)j * (MAXM + 1);
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) col[i] = colL[i];
}

__global__ void k_arnoldi_start(ArnoldiState* st, int nblk, const double* __restrict__ npart) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += npart[b];
  s = block_sum(s, sh);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(s);
  for (int i = 0; i <= MAXM; ++i) st->g[i] = 0.0;
  st->g[0] = beta;
  st->resid = beta;
  st->inv_hnext = beta > 0 ? 1.0 / beta : 0.0;
}

// back substitution H(0:k,0:k) y = g(0:k)
// y = R^-1 g on the rotated Hessenberg.  A zero diagonal (a breakdown column
// whose direction the basis already spans; in flexible GMRES H may be singular)
// drops that direction instead of dividing by zero; the true residual computed
// after the update decides whether the cycle converged.
// Column-oriented, one work-group: y_i = g_i / R_ii, then g_c -= R_ci y_i for
// c < i by all threads (column i of R is contiguous).
__global__ void k_backsolve(ArnoldiState* st, int k) {
  if (blockIdx.x != 0) return;
  __shared__ double gs[MAXM];
  const int ld = MAXM + 1;
  for (int i = threadIdx.x; i < k; i += blockDim.x) gs[i] = st->g[i];
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    const double* col = st->H + (int64_t)i * ld;
    const double d = col[i];
    const double yi = d != 0.0 ? gs[i] / d : 0.0;
    for (int c = threadIdx.x; c < i; c += blockDim.x) gs[c] -= col[c] * yi;
    if (threadIdx.x == 0) st->y[i] = yi;
    __syncthreads();
  }
}

// ------------------------------------------- delayed re-orthogonalization ---
// Flexible GMRES with classical Gram-Schmidt whose second (re-orthogonalization)
// pass is delayed by one step and folded into the next step's sweeps, so that
// each Arnoldi step reads the basis twice instead of three times.  At step j,
// U is the previous step's once-orthogonalized, unnormalized vector and
// W = A z_j with z_j = M(U) (FGMRES allows any z_j as long as A z_j is expanded
// in the final orthonormal basis):
//   sweep 1 (k_dc_dots):   a = V^T U, b = V^T W, U.U, U.W, W.W     (V = v_0..v_{j-1})
//   scalars (k_dc_scalar): s = a, alpha = sqrt(U.U - |s|^2), v_j = (U - V s)/alpha,
//                          column j-1 of H = [h1_{j-1} + s ; alpha] -> Givens,
//                          h1_j = [b ; c], c = v_j.W = (U.W - s.b)/alpha
//   sweep 2 (k_dc_update): v_j = (U - V s)/alpha, U <- W - V h1_j
//                          = W - (c/alpha) U - V (b - (c/alpha) s)
// Column j-1 of H is final one step late; a closing sweep 1 (without W) finalizes
// the last column of a cycle.  At j = 0, U = r and alpha = ||r|| (g_0 = alpha).

// rows of part: [0, j) U.V_i, [j, 2j) W.V_i, 2j U.U, 2j+1 U.W, 2j+2 W.W (W nullable)
template <int G>
__global__ void __launch_bounds__(VB) k_dc_dots(int64_t n, int j, const double* __restrict__ V, int64_t ldv,
                                                const double* __restrict__ U, const double* __restrict__ W,
                                                double* __restrict__ part) {
  __shared__ double sh[VB / 64][2 * G + 3];
  int64_t lo, hi;
  chunk_of(n, &lo, &hi);
  const int nblk = gridDim.x;
  const bool hw = W != nullptr;
  const int ngroups = j > 0 ? (j + G - 1) / G : 1;
  for (int gi = 0; gi < ngroups; ++gi) {
    const int i0 = gi * G;
    const int ni = j - i0 < G ? (j - i0 > 0 ? j - i0 : 0) : G;
    double s[2 * G + 3];
#pragma unroll
    for (int r = 0; r < 2 * G + 3; ++r) s[r] = 0.0;
    for (int64_t t = lo + threadIdx.x; t < hi; t += VB) {
      const double ut = U[t];
      const double wt = hw ? W[t] : 0.0;
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const double v = (r < ni) ? V[(int64_t)(i0 + r) * ldv + t] : 0.0;
        s[r] += v * ut;
        s[G + r] += v * wt;
      }
      s[2 * G] += ut * ut;
      s[2 * G + 1] += ut * wt;
      s[2 * G + 2] += wt * wt;
    }
    const double tot = block_sum_many<2 * G + 3>(s, 2 * G + 3, sh);
    const int q = threadIdx.x;
    int row = -1;
    if (q < G) {
      if (q < ni) row = i0 + q;
    } else if (q < 2 * G) {
      if (q - G < ni) row = j + i0 + (q - G);
    } else if (q < 2 * G + 3 && gi == 0) {
      row = 2 * j + (q - 2 * G);
    }
    if (row >= 0) part[(int64_t)row * nblk + blockIdx.x] = tot;
  }
}

// coefficient block of sweep 2: [0, MAXM) s, [MAXM, 2 MAXM) gamma, 2 MAXM: 1/alpha, 2 MAXM + 1: c/alpha
constexpr int DC_COEF = 2 * MAXM + 2;

// One work-group of 1024 threads.  The block partials of sweep 1 (rows laid out
// as by k_dc_dots, nblk partials each) are first reduced into LDS, one row per
// wave at a time (fixed order: deterministic); thread 0 then does the sequential part;
// the coefficient writes are spread over the threads.  h1p holds h1_{j-1} on
// entry and h1_j on exit.
constexpr int DC_SCALAR_THREADS = 1024;
__global__ void __launch_bounds__(DC_SCALAR_THREADS) k_dc_scalar(ArnoldiState* st, int j, int closing,
                                                  const double* __restrict__ part, int nblk,
                                                  double* __restrict__ h1p, double* __restrict__ coef) {
  __shared__ double dots[2 * MAXM + 3];
  __shared__ double colL[MAXM + 1], csL[MAXM], snL[MAXM];
  __shared__ double red[2][DC_SCALAR_THREADS / 64];
  __shared__ double bc[3];   // 1/alpha, c/alpha, c
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int row = wid; row < 2 * j + 3; row += nw) {
    double v = 0.0;
#pragma unroll 8
    for (int b = lane; b < nblk; b += 64) v += part[(int64_t)row * nblk + b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) dots[row] = v;
  }
  __syncthreads();
  const double* a = dots;
  const double* b = dots + j;
  // a.a and a.b over the work-group; the new Hessenberg column and the previous
  // rotations staged in LDS for the sequential rotation chain of thread 0
  {
    double pa = 0.0, pb = 0.0;
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
      pa += a[i] * a[i];
      pb += a[i] * b[i];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      pa += __shfl_down(pa, off, 64);
      pb += __shfl_down(pb, off, 64);
    }
    if (lane == 0) {
      red[0][wid] = pa;
      red[1][wid] = pb;
    }
  }
  // U holds the pending vector divided by sigma (the previous step's alpha), which keeps
  // its magnitude from compounding over the cycle; the column takes the factor back
  const double sg = j > 0 ? st->sigma : 1.0;
  for (int i = threadIdx.x; i < j; i += blockDim.x) colL[i] = h1p[i] + sg * a[i];
  for (int i = threadIdx.x; i + 1 < j; i += blockDim.x) {
    csL[i] = st->cs[i];
    snL[i] = st->sn[i];
  }
  if (j == 0)
    for (int i = threadIdx.x; i <= MAXM; i += blockDim.x) st->g[i] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double uu = dots[2 * j], uw = dots[2 * j + 1], ww = dots[2 * j + 2];
    double ss = 0.0, sb = 0.0;
    for (int w = 0; w < nw; ++w) {
      ss += red[0][w];
      sb += red[1][w];
    }
    double al2 = uu - ss;
    const double al = al2 > 0.0 ? sqrt(al2) : 0.0;
    int brk = 0;
    if (j == 0) {
      st->g[0] = al;
      st->resid = al;
    } else {
      const int c = j - 1;
      colL[j] = sg * al;
      brk = (sg * al <= 1e-14 * st->wnorm0) ? 1 : 0;
      for (int i = 0; i < c; ++i) {
        const double t = csL[i] * colL[i] + snL[i] * colL[i + 1];
        colL[i + 1] = -snL[i] * colL[i] + csL[i] * colL[i + 1];
        colL[i] = t;
      }
      const double d = hypot(colL[c], colL[c + 1]);
      st->cs[c] = d > 0 ? colL[c] / d : 1.0;
      st->sn[c] = d > 0 ? colL[c + 1] / d : 0.0;
      colL[c] = d;
      colL[c + 1] = 0.0;
      st->g[c + 1] = -st->sn[c] * st->g[c];
      st->g[c] = st->cs[c] * st->g[c];
      st->resid = fabs(st->g[c + 1]);
    }
    st->breakdown = brk;
    const double inva = (al > 0.0 && !brk) ? 1.0 / al : 0.0;
    const double cc = (uw - sb) * inva;
    bc[0] = inva;
    bc[1] = cc * inva;
    bc[2] = cc;
    if (!closing) st->wnorm0 = sqrt(ww);
    st->sigma = al;   // the next pending vector is divided by this alpha (k_dc_update)
  }
  __syncthreads();
  if (j > 0) {
    double* col = st->H + (int64_t)(j - 1) * (MAXM + 1);
    for (int i = threadIdx.x; i <= j; i += blockDim.x) col[i] = colL[i];
  }
  if (closing) return;
  const double dl = bc[1];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    coef[i] = a[i];
    coef[MAXM + i] = b[i] - dl * a[i];
    h1p[i] = b[i];
  }
  if (threadIdx.x == 0) {
    h1p[j] = bc[2];
    coef[2 * MAXM] = bc[0];
    coef[2 * MAXM + 1] = dl;
  }
}

// v_j = (U - V s)/alpha -> Vj ; U <- (W - (c/alpha) U - V gamma) / alpha
// (the division keeps the pending vector's magnitude from growing by |J M| per
// step over a long cycle; k_dc_scalar multiplies the next column back)
template <int G>
__global__ void __launch_bounds__(VB) k_dc_update(int64_t n, int j, const double* __restrict__ V, int64_t ldv,
                                                  const double* __restrict__ coef, double* __restrict__ U,
                                                  const double* __restrict__ W, double* __restrict__ Vj) {
  __shared__ double cs_[2 * MAXM + 2];
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    cs_[i] = coef[i];
    cs_[MAXM + i] = coef[MAXM + i];
  }
  if (threadIdx.x == 0) {
    cs_[2 * MAXM] = coef[2 * MAXM];
    cs_[2 * MAXM + 1] = coef[2 * MAXM + 1];
  }
  __syncthreads();
  const double inva = cs_[2 * MAXM], dl = cs_[2 * MAXM + 1];
  int64_t lo, hi;
  chunk_of(n, &lo, &hi);
  for (int64_t t = lo + threadIdx.x; t < hi; t += VB) {
    const double ut = U[t];
    double va = ut, ua = W[t] - dl * ut;
    for (int i0 = 0; i0 < j; i0 += G) {
      double v[G];
#pragma unroll
      for (int r = 0; r < G; ++r) v[r] = (i0 + r < j) ? V[(int64_t)(i0 + r) * ldv + t] : 0.0;
#pragma unroll
      for (int r = 0; r < G; ++r) {
        if (i0 + r < j) {
          va -= cs_[i0 + r] * v[r];
          ua -= cs_[MAXM + i0 + r] * v[r];
        }
      }
    }
    Vj[t] = va * inva;
    U[t] = ua * inva;
  }
}

__global__ void k_to_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

// NaN injection for the failure-handling tests
__global__ void k_poison(int64_t n, double* z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (i % 97) == 0) z[i] = __longlong_as_double(0x7ff8000000000000ll);
}

}  // namespace ldg

using namespace ldg;

struct ldg_precond_s;
namespace ldg {
ldg_status precond_apply_impl(ldg_precond_s* pc, const double* r, double* z, hipStream_t s);
ldg_status precond_apply_impl32(ldg_precond_s* pc, const double* r, float* z, hipStream_t s);
ldg_status precond_rebuild(ldg_precond_s* pc, const ldg_time* t, const double* u_lin, hipStream_t s);
int precond_kind(const ldg_precond_s* pc);
ldg_precond_s* precond_fallback(ldg_precond_s* pc);
ldg_status precond_count_nonfinite(ldg_precond_s* pc, const double* z, int64_t n, int* host_cnt, hipStream_t s);
}

namespace {

struct Workspace {
  int64_t n = 0;
  int m = 0;
  double* V = nullptr;     // [(m+1)][n]
  double* Z = nullptr;     // [m][n] (FP64 solves)
  float* Z32 = nullptr;    // [m][n] (FP32-state solves, instead of Z)
  float* u32 = nullptr;    // [n] FP32 copy of the linearization point (FP32-state solves)
  bool s32 = false;
  double* w = nullptr;
  double* r = nullptr;
  double* part = nullptr;  // [(2 MAXM + 3) * RED_BLOCKS] block partials
  double* npart = nullptr; // [RED_BLOCKS]
  double* h1 = nullptr;
  double* h2 = nullptr;
  double* U = nullptr;     // delayed re-orthogonalization: the pending vector
  double* coef = nullptr;  // [DC_COEF]
  ArnoldiState* st = nullptr;
  double* pinned = nullptr;  // host scalars
  hipEvent_t ev[8];        // phase timing events of the sampled steps, two slots of four
  hipEvent_t evs[2];       // step-end events of the other steps (no timing)
  bool ok = false;
  void release() {
    if (!ok) return;
    hipFree(V); hipFree(Z); hipFree(Z32); hipFree(u32); hipFree(w); hipFree(r); hipFree(part); hipFree(npart);
    hipFree(h1); hipFree(h2);
    Z = nullptr; Z32 = nullptr; u32 = nullptr;
    hipFree(U); hipFree(coef);
    hipFree(st); hipHostFree(pinned);
    for (auto& e : ev) hipEventDestroy(e);
    for (auto& e : evs) hipEventDestroy(e);
    ok = false;
  }
  ldg_status ensure(int64_t nn, int mm, bool state32) {
    if (ok && nn == n && mm <= m && state32 == s32) return LDG_OK;
    release();
    n = nn; m = mm; s32 = state32;
    LDG_TRY(hipMalloc((void**)&V, sizeof(double) * (m + 1) * n));
    if (s32) {
      LDG_TRY(hipMalloc((void**)&Z32, sizeof(float) * m * n));
      LDG_TRY(hipMalloc((void**)&u32, sizeof(float) * n));
    } else {
      LDG_TRY(hipMalloc((void**)&Z, sizeof(double) * m * n));
    }
    LDG_TRY(hipMalloc((void**)&w, sizeof(double) * n));
    LDG_TRY(hipMalloc((void**)&r, sizeof(double) * n));
    LDG_TRY(hipMalloc((void**)&part, sizeof(double) * (2 * MAXM + 3) * RED_BLOCKS));
    LDG_TRY(hipMalloc((void**)&npart, sizeof(double) * RED_BLOCKS));
    LDG_TRY(hipMalloc((void**)&h1, sizeof(double) * (MAXM + 1)));
    LDG_TRY(hipMalloc((void**)&h2, sizeof(double) * (MAXM + 1)));
    LDG_TRY(hipMalloc((void**)&U, sizeof(double) * n));
    LDG_TRY(hipMalloc((void**)&coef, sizeof(double) * DC_COEF));
    LDG_TRY(hipMalloc((void**)&st, sizeof(ArnoldiState)));
    LDG_TRY(hipHostMalloc((void**)&pinned, sizeof(double) * 8, hipHostMallocDefault));
    for (auto& e : ev) LDG_TRY(hipEventCreate(&e));
    for (auto& e : evs) LDG_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ok = true;
    return LDG_OK;
  }
};

// per-thread solver workspace, kept until the process ends
thread_local Workspace* g_ws_ptr = nullptr;

// Phase times (preconditioner, JVP, orthogonalization) are taken with timing
// events on every PHASE_SAMPLE-th Arnoldi step only and scaled to all steps:
// each timing event record left the GPU idle for 5-10 us, about 8% of a step.
// The other steps record one event without timing for the host's wait.
constexpr int PHASE_SAMPLE = 8;

struct PhaseClock {
  double pc = 0.0, jvp = 0.0, orth = 0.0;
  int64_t timed = 0, steps = 0;
  bool slot_timed[2] = {false, false};
  // before queuing a step into slot sl
  bool begin(int its, int sl) { return slot_timed[sl] = (its % PHASE_SAMPLE) == 0; }
  void mark(Workspace& ws, int sl, int k, hipStream_t s) const {
    if (slot_timed[sl]) hipEventRecord(ws.ev[4 * sl + k], s);
  }
  void end(Workspace& ws, int sl, hipStream_t s) const {
    hipEventRecord(slot_timed[sl] ? ws.ev[4 * sl + 3] : ws.evs[sl], s);
  }
  // wait for the step in slot sl and account for it
  bool wait(Workspace& ws, int sl) {
    if (hipEventSynchronize(slot_timed[sl] ? ws.ev[4 * sl + 3] : ws.evs[sl]) != hipSuccess) return false;
    ++steps;
    if (slot_timed[sl]) {
      float ms = 0.0f;
      ++timed;
      if (hipEventElapsedTime(&ms, ws.ev[4 * sl + 0], ws.ev[4 * sl + 1]) == hipSuccess) pc += ms * 1e-3;
      if (hipEventElapsedTime(&ms, ws.ev[4 * sl + 1], ws.ev[4 * sl + 2]) == hipSuccess) jvp += ms * 1e-3;
      if (hipEventElapsedTime(&ms, ws.ev[4 * sl + 2], ws.ev[4 * sl + 3]) == hipSuccess) orth += ms * 1e-3;
    }
    return true;
  }
  void report(ldg_gmres_stats& S) const {
    const double f = timed ? double(steps) / double(timed) : 0.0;
    S.t_pc = pc * f;
    S.t_jvp = jvp * f;
    S.t_orth = orth * f;
  }
};

inline int nblk_for(int64_t n) {
  int64_t g = (n + VB - 1) / VB;
  return (int)(g > RED_BLOCKS ? RED_BLOCKS : (g < 1 ? 1 : g));
}

}  // namespace

namespace ldg {

// The three CGS2 sweeps.  Register tiles: the dot sweep keeps at most 16
// accumulators (more cost occupancy than they save in re-reads of w), the
// update-only sweep reads the basis 8 vectors at a time, and the fused
// update + dot sweep keeps all nv <= 32 basis values of an element index live.
// At most 512 work-groups: fewer, longer chunks measured faster for these
// streaming sweeps.
template <int GB>
static void cgs2_launch(int64_t n, int nv, int nb, Workspace& ws, hipStream_t s) {
  if (nv <= 8) hipLaunchKernelGGL((k_cgs_dots<8>), dim3(nb), dim3(VB), 0, s, n, nv, ws.V, n, ws.w, ws.part);
  else hipLaunchKernelGGL((k_cgs_dots<16>), dim3(nb), dim3(VB), 0, s, n, nv, ws.V, n, ws.w, ws.part);
  hipLaunchKernelGGL(k_reduce_rows, dim3(nv + 1), dim3(VB), 0, s, nv + 1, nb, ws.part, ws.h1);
  if (nv <= GB) {
    hipLaunchKernelGGL((k_cgs_update_dots<GB>), dim3(nb), dim3(VB), 0, s, n, nv, ws.V, n, ws.h1, ws.w, ws.part);
  } else {
    hipLaunchKernelGGL((k_cgs_update<8>), dim3(nb), dim3(VB), 0, s, n, nv, ws.V, n, ws.h1, ws.w, (double*)nullptr);
    hipLaunchKernelGGL((k_cgs_dots<16>), dim3(nb), dim3(VB), 0, s, n, nv, ws.V, n, ws.w, ws.part);
  }
  hipLaunchKernelGGL(k_reduce_rows, dim3(nv), dim3(VB), 0, s, nv, nb, ws.part, ws.h2);
  hipLaunchKernelGGL((k_cgs_update<8>), dim3(nb), dim3(VB), 0, s, n, nv, ws.V, n, ws.h2, ws.w, ws.npart);
}

inline int cgs_blocks(int64_t n) { return std::min(nblk_for(n), 512); }

static ldg_status cgs2(int64_t n, int nv, Workspace& ws, hipStream_t s) {
  const int nb = cgs_blocks(n);
  if (nv <= 8) cgs2_launch<8>(n, nv, nb, ws, s);
  else if (nv <= 16) cgs2_launch<16>(n, nv, nb, ws, s);
  else cgs2_launch<32>(n, nv, nb, ws, s);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

// Modified Gram-Schmidt (one pass): for i = 0..nv-1, h1_i = V_i . w, w -= h1_i V_i.
// Leaves h2 = 0, h1[nv] = ||w||^2 before the orthogonalization and the block
// partials of the final ||w||^2 in npart, as the CGS2 path does.
static ldg_status mgs(int64_t n, int nv, Workspace& ws, hipStream_t s) {
  const int nb = cgs_blocks(n);
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(VB), 0, s, (int64_t)(MAXM + 1), 0.0, ws.h2);
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(VB), 0, s, n, ws.w, ws.w, ws.part);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(VB), 0, s, nb, ws.part, ws.h1 + nv);
  for (int i = 0; i < nv; ++i) {
    const double* vi = ws.V + (int64_t)i * n;
    hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(VB), 0, s, n, vi, ws.w, ws.part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(VB), 0, s, nb, ws.part, ws.h1 + i);
    hipLaunchKernelGGL(k_axmy_dev, dim3(nb), dim3(VB), 0, s, n, ws.h1 + i, vi, ws.w);
  }
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(VB), 0, s, n, ws.w, ws.w, ws.npart);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

// w = b - J x  -> ws.r ; returns ||r|| on the host
static ldg_status true_residual(Model& md, const ldg_time* t, const double* u, const double* b, const double* x,
                                ldg_precision prec, Workspace& ws, double* out_norm, hipStream_t s) {
  ldg_status st = jvp_impl(md, t, u, x, ws.r, prec == LDG_JVP_FD ? LDG_JVP_FD : LDG_FP64, true, s);
  if (st != LDG_OK) return st;
  st = vec_axpby(ws.n, 1.0, b, -1.0, ws.r, s);
  if (st != LDG_OK) return st;
  double nr = 0.0;
  st = vec_norm2(ws.n, ws.r, ws.part, &nr, s);
  *out_norm = std::sqrt(nr);
  return st;
}

// One restart cycle of FGMRES with the delayed re-orthogonalization (orth = 2):
// k returns the number of final columns of H, stop whether the cycle ended on
// convergence or breakdown.  ws.r holds the cycle's residual on entry.
// Training-data hook (ldg_gmres_opts.record_*): the preconditioner's input v
// of global step `its` and the product J z of its output, copied for the caller.
static ldg_status record_pair(const ldg_gmres_opts& o, int its, int64_t n, const double* vj, const double* jz,
                              hipStream_t s) {
  if (!o.record_v || its >= o.record_max) return LDG_OK;
  LDG_TRY(hipMemcpyAsync(o.record_v + (int64_t)its * n, vj, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  LDG_TRY(hipMemcpyAsync(o.record_jz + (int64_t)its * n, jz, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  return LDG_OK;
}

static ldg_status dcgs2_cycle(Model& md, const ldg_time* t, const double* u_lin, ldg_precision jp,
                              const ldg_gmres_opts& o, Workspace& ws, ldg_precond_s*& pc_cur, bool watch, int watch_win,
                              double& watch_ref, int& watch_it, double tol, int& its, int& k, bool& stop,
                              ldg_status& result, ldg_gmres_stats& S, PhaseClock& clk, hipStream_t s) {
  const int64_t n = ws.n;
  const int m = o.restart;
  const int nbc = cgs_blocks(n);
  const bool use_pc = o.pc != nullptr;
  const bool pipelined = !watch;
  ldg_status st;
  LDG_TRY(hipMemcpyAsync(ws.U, ws.r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  // sweep 1 (block partials; k_dc_scalar reduces them)
  auto sweep1 = [&](int j, const double* Wp) {
    if (j <= 8) hipLaunchKernelGGL((k_dc_dots<8>), dim3(nbc), dim3(VB), 0, s, n, j, ws.V, n, ws.U, Wp, ws.part);
    else hipLaunchKernelGGL((k_dc_dots<16>), dim3(nbc), dim3(VB), 0, s, n, j, ws.V, n, ws.U, Wp, ws.part);
  };
  // read step jj's result: after it, columns 0..jj-1 of H are final
  auto finish = [&](int jj) -> bool {
    const int sl = jj & 1;
    if (!clk.wait(ws, sl)) {
      result = LDG_EDEVICE;
      set_error("event synchronization failed");
      return true;
    }
    k = jj;
    if (jj == 0) return false;
    const double res = ws.pinned[2 * sl];
    int brk = 0;
    std::memcpy(&brk, ws.pinned + 2 * sl + 1, sizeof(int));
    S.res_est = res;
    if (!std::isfinite(res)) { result = LDG_EBREAKDOWN; return true; }
    if (watch && watch_win > 0 && pc_cur == o.pc) {
      if (watch_ref < 0) { watch_ref = res; watch_it = 0; }
      if (++watch_it >= watch_win) {
        if (res > 0.99 * watch_ref && precond_fallback(o.pc)) { pc_cur = precond_fallback(o.pc); S.fell_back = 1; }
        watch_ref = res;
        watch_it = 0;
      }
    }
    return res <= tol || brk;
  };
  int queued = -1, done = 0;
  const bool s32 = o.state32 != 0;
  for (int j = 0; j < m && its < o.maxit; ++j) {
    const int sl = j & 1;
    double* zj = s32 ? nullptr : ws.Z + (int64_t)j * n;
    float* zj32 = s32 ? ws.Z32 + (int64_t)j * n : nullptr;
    clk.begin(its, sl);
    clk.mark(ws, sl, 0, s);
    if (s32) {
      // FP32 state: z_j stored in FP32, the product reads it and the FP32 copy of u_lin
      if (use_pc) {
        st = precond_apply_impl32(pc_cur, ws.U, zj32, s);
        if (st != LDG_OK) return st;
      } else {
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(VB), 0, s, n, ws.U, zj32);
      }
    } else if (use_pc) {
      st = precond_apply_impl(pc_cur, ws.U, zj, s);
      if (st != LDG_OK) return st;
      if (o.inject_fault == 1) hipLaunchKernelGGL(k_poison, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, zj);
      if (watch && pc_cur == o.pc) {
        int bad = 0;
        st = precond_count_nonfinite(pc_cur, zj, n, &bad, s);
        if (st != LDG_OK) return st;
        if (bad) {
          ldg_precond_s* fb = precond_fallback(o.pc);
          if (!fb) { result = LDG_EBREAKDOWN; break; }
          pc_cur = fb;
          S.fell_back = 1;
          st = precond_apply_impl(pc_cur, ws.U, zj, s);
          if (st != LDG_OK) return st;
        }
      }
    } else {
      LDG_TRY(hipMemcpyAsync(zj, ws.U, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    clk.mark(ws, sl, 1, s);
    st = s32 ? jvp_state32(md, t, ws.u32, zj32, ws.w, true, s) : jvp_impl(md, t, u_lin, zj, ws.w, jp, true, s);
    if (st != LDG_OK) return st;
    if (!s32 && (st = record_pair(o, its, n, ws.U, ws.w, s)) != LDG_OK) return st;
    clk.mark(ws, sl, 2, s);
    sweep1(j, ws.w);
    hipLaunchKernelGGL(k_dc_scalar, dim3(1), dim3(DC_SCALAR_THREADS), 0, s, ws.st, j, 0, ws.part, nbc, ws.h1, ws.coef);
    if (j <= 8)
      hipLaunchKernelGGL((k_dc_update<8>), dim3(nbc), dim3(VB), 0, s, n, j, ws.V, n, ws.coef, ws.U, ws.w,
                         ws.V + (int64_t)j * n);
    else
      hipLaunchKernelGGL((k_dc_update<16>), dim3(nbc), dim3(VB), 0, s, n, j, ws.V, n, ws.coef, ws.U, ws.w,
                         ws.V + (int64_t)j * n);
    LDG_TRY(hipGetLastError());
    LDG_TRY(hipMemcpyAsync(ws.pinned + 2 * sl, &ws.st->resid, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    clk.end(ws, sl, s);
    ++its;
    done = j + 1;
    if (!pipelined) {
      if (finish(j)) { stop = true; break; }
      continue;
    }
    const int prev = queued;
    queued = j;
    if (prev >= 0 && finish(prev)) {
      // step j was queued past the end of the cycle: not counted
      --its;
      queued = -1;
      stop = true;
      break;
    }
  }
  if (queued >= 0 && result == LDG_OK) stop = finish(queued);
  if (result != LDG_OK) return LDG_OK;
  if (!stop && done > 0) {
    // close the cycle: re-orthogonalize the pending vector to finalize column done-1
    sweep1(done, nullptr);
    hipLaunchKernelGGL(k_dc_scalar, dim3(1), dim3(DC_SCALAR_THREADS), 0, s, ws.st, done, 1, ws.part, nbc, ws.h1, ws.coef);
    LDG_TRY(hipGetLastError());
    LDG_TRY(hipMemcpyAsync(ws.pinned, &ws.st->resid, sizeof(double), hipMemcpyDeviceToHost, s));
    LDG_TRY(hipStreamSynchronize(s));
    k = done;
    S.res_est = ws.pinned[0];
    if (!std::isfinite(S.res_est)) result = LDG_EBREAKDOWN;
  }
  return LDG_OK;
}

ldg_status gmres_impl(Model& md, const ldg_time* t, const double* u_lin, const double* b, double* x,
                      const ldg_gmres_opts& o, ldg_gmres_stats* stats, hipStream_t s) {
  auto T0 = std::chrono::steady_clock::now();
  ldg_gmres_stats S{};
  const int64_t n = (int64_t)md.N();
  const int m = o.restart;
  if (m < 1 || m > MAXM) { set_error("restart must be in [1, " + std::to_string(MAXM) + "]"); return LDG_EINVAL; }
  if (o.orth < 0 || o.orth > 2) { set_error("orth must be 0 (CGS2), 1 (MGS) or 2 (delayed CGS2)"); return LDG_EINVAL; }
  if (o.state32) {
    if (o.jvp_prec != LDG_FP32) { set_error("state32 needs jvp_prec = LDG_FP32"); return LDG_EINVAL; }
    if (o.orth != 2) { set_error("state32 is built for the delayed CGS2 orthogonalization (orth = 2)"); return LDG_EUNSUPPORTED; }
  }
  if ((o.record_v != nullptr) != (o.record_jz != nullptr) || o.record_max < 0) {
    set_error("record_v and record_jz are given together, with record_max >= 0");
    return LDG_EINVAL;
  }
  if (o.record_v && o.state32) { set_error("recording is not built for the FP32 state"); return LDG_EUNSUPPORTED; }
  if (!g_ws_ptr) g_ws_ptr = new Workspace();
  Workspace& ws = *g_ws_ptr;
  ldg_status st = ws.ensure(n, m, o.state32 != 0);
  if (st != LDG_OK) return st;
  const int nb = nblk_for(n);
  const int gV = nb;
  // linearization point: q(u_lin) for the nonlinear models, once per solve
  if (!md.linear && md.hasq) {
    md.q_of[1] = nullptr;
    st = form_q_cache64(md, u_lin, s);
    if (st != LDG_OK) return st;
    if (o.jvp_prec == LDG_FP32) {
      st = form_q_cache32(md, u_lin, PM_FP32, s);
      if (st != LDG_OK) return st;
    }
  }
  if (o.state32 && u_lin) hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(VB), 0, s, n, u_lin, ws.u32);
  const ldg_precision jp = o.jvp_prec;
  const bool use_pc = o.pc != nullptr;
  // learned preconditioner: watched for non-finite output and stagnation
  // (residual estimate reduced by less than 1% over watch_win iterations: one
  // restart cycle unless the caller sets it; none when negative); then block-Jacobi
  ldg_precond_s* pc_cur = o.pc;
  const bool watch = use_pc && precond_kind(o.pc) == 1;
  const int watch_win = o.watch_window > 0 ? o.watch_window : (o.watch_window == 0 ? m : 0);
  double watch_ref = -1.0;
  int watch_it = 0;
  double r0 = 0.0;
  st = true_residual(md, t, u_lin, b, x, jp, ws, &r0, s);
  if (st != LDG_OK) return st;
  S.res0 = r0;
  const double tol = std::max(o.rtol * r0, o.atol);
  double beta = r0;
  int its = 0;
  ldg_status result = LDG_OK;
  PhaseClock clk;
  while (beta > tol && its < o.maxit) {
    if (!std::isfinite(beta)) { result = LDG_EBREAKDOWN; break; }
    int k = 0;
    bool stop = false;
    if (o.orth == 2) {
      st = dcgs2_cycle(md, t, u_lin, jp, o, ws, pc_cur, watch, watch_win, watch_ref, watch_it, tol, its, k, stop, result, S, clk, s);
      if (st != LDG_OK) return st;
      if (result == LDG_EDEVICE) return result;
    } else {
      // V0 = r / beta
      hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(VB), 0, s, n, ws.r, ws.r, ws.npart);
      hipLaunchKernelGGL(k_arnoldi_start, dim3(1), dim3(VB), 0, s, ws.st, nb, ws.npart);
      hipLaunchKernelGGL(k_scale_dev, dim3(gV), dim3(VB), 0, s, n, &ws.st->inv_hnext, ws.r, ws.V);
      // Without the learned preconditioner's host-side watch, step j + 1 is queued
      // before the host reads step j's residual estimate, so the GPU never waits for
      // the host.  A queued step after convergence or breakdown only touches
      // column j + 1 of H, g[j + 1..j + 2] and V[j + 2]; the solution update uses
      // the first k columns only (a step after a breakdown works on a zero vector).
      const bool pipelined = !watch;
      int queued = -1;                  // last queued step whose result is unread
      // read step jj's result (slot jj & 1); true when the cycle ends there
      auto finish = [&](int jj) -> bool {
        const int sl = jj & 1;
        if (!clk.wait(ws, sl)) { result = LDG_EDEVICE; set_error("event synchronization failed"); return true; }
        k = jj + 1;
        const double res = ws.pinned[2 * sl];
        int brk = 0;
        std::memcpy(&brk, ws.pinned + 2 * sl + 1, sizeof(int));
        S.res_est = res;
        if (!std::isfinite(res)) { result = LDG_EBREAKDOWN; return true; }
        if (watch && watch_win > 0 && pc_cur == o.pc) {
          if (watch_ref < 0) { watch_ref = res; watch_it = 0; }
          if (++watch_it >= watch_win) {
            if (res > 0.99 * watch_ref && precond_fallback(o.pc)) { pc_cur = precond_fallback(o.pc); S.fell_back = 1; }
            watch_ref = res;
            watch_it = 0;
          }
        }
        return res <= tol || brk;
      };
      for (int j = 0; j < m && its < o.maxit; ++j) {
        const int sl = j & 1;
        double* vj = ws.V + (int64_t)j * n;
        double* zj = use_pc ? ws.Z + (int64_t)j * n : vj;
        clk.begin(its, sl);
        clk.mark(ws, sl, 0, s);
        if (use_pc) {
          st = precond_apply_impl(pc_cur, vj, zj, s);
          if (st != LDG_OK) return st;
          if (o.inject_fault == 1) hipLaunchKernelGGL(k_poison, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, zj);
          if (watch && pc_cur == o.pc) {
            int bad = 0;
            st = precond_count_nonfinite(pc_cur, zj, n, &bad, s);
            if (st != LDG_OK) return st;
            if (bad) {
              ldg_precond_s* fb = precond_fallback(o.pc);
              if (!fb) { result = LDG_EBREAKDOWN; break; }
              pc_cur = fb;
              S.fell_back = 1;
              st = precond_apply_impl(pc_cur, vj, zj, s);
              if (st != LDG_OK) return st;
            }
          }
        }
        clk.mark(ws, sl, 1, s);
        st = jvp_impl(md, t, u_lin, zj, ws.w, jp, true, s);
        if (st != LDG_OK) return st;
        if ((st = record_pair(o, its, n, vj, ws.w, s)) != LDG_OK) return st;
        clk.mark(ws, sl, 2, s);
        // CGS2: h1 = V^T w (+ ||w||^2), w -= V h1, h2 = V^T w, w -= V h2 (+ ||w||^2); or MGS
        st = o.orth == 1 ? mgs(n, j + 1, ws, s) : cgs2(n, j + 1, ws, s);
        if (st != LDG_OK) return st;
        hipLaunchKernelGGL(k_givens, dim3(1), dim3(VB), 0, s, ws.st, j, cgs_blocks(n), ws.h1, ws.h2, ws.npart);
        hipLaunchKernelGGL(k_scale_dev, dim3(gV), dim3(VB), 0, s, n, &ws.st->inv_hnext, ws.w,
                           ws.V + (int64_t)(j + 1) * n);
        LDG_TRY(hipGetLastError());
        LDG_TRY(hipMemcpyAsync(ws.pinned + 2 * sl, &ws.st->resid, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        clk.end(ws, sl, s);
        ++its;
        if (!pipelined) {
          if (finish(j)) { stop = true; break; }
          continue;
        }
        const int prev = queued;
        queued = j;
        if (prev >= 0 && finish(prev)) {
          // step j was queued past the end of the cycle: not counted
          --its;
          queued = -1;
          stop = true;
          break;
        }
      }
      if (queued >= 0 && result == LDG_OK) stop = finish(queued);
      if (result == LDG_EDEVICE) return result;
    }
    // x += Z y
    if (k > 0 && result == LDG_OK) {
      hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(256), 0, s, ws.st, k);
      if (o.state32)
        hipLaunchKernelGGL(k_combine<float>, dim3(gV), dim3(VB), 0, s, n, k, (const float*)ws.Z32, n, ws.st->y, x);
      else
        hipLaunchKernelGGL(k_combine<double>, dim3(gV), dim3(VB), 0, s, n, k,
                           (const double*)((use_pc || o.orth == 2) ? ws.Z : ws.V), n, ws.st->y, x);
      LDG_TRY(hipGetLastError());
    }
    ++S.restarts;
    if (result != LDG_OK) break;
    st = true_residual(md, t, u_lin, b, x, jp, ws, &beta, s);
    if (st != LDG_OK) return st;
    (void)stop;
  }
  S.iters = its;
  S.res_true = beta;
  if (result == LDG_OK && !(beta <= tol * (1.0 + 1e-6) || beta <= tol)) {
    // Givens estimate met the tolerance but the true residual did not, or maxit reached
    result = LDG_ENOCONV;
  }
  if (!std::isfinite(beta)) result = LDG_EBREAKDOWN;
  clk.report(S);
  S.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - T0).count();
  if (stats) *stats = S;
  if (result == LDG_ENOCONV) set_error("GMRES did not reach the tolerance");
  if (result == LDG_EBREAKDOWN) set_error("non-finite value in GMRES");
  return result;
}

}  // namespace ldg


extern "C" {

ldg_status ldg_gmres_solve(ldg_model md, const ldg_time* t, const double* u_lin, const double* b, double* x,
                           const ldg_gmres_opts* opts, ldg_gmres_stats* stats, void* stream) {
  LDG_ENTER();
  if (!md || !b || !x || !opts) { set_error("null argument"); return LDG_EINVAL; }
  if (!md->linear && !u_lin) { set_error("nonlinear model needs u_lin"); return LDG_EINVAL; }
  return gmres_impl(*md, t, u_lin, b, x, *opts, stats, (hipStream_t)stream);
}

ldg_status ldg_newton_solve(ldg_model md, const ldg_time* t, double* u, const ldg_newton_opts* opts,
                            ldg_newton_stats* stats, void* stream) {
  LDG_ENTER();
  if (!md || !u || !opts) { set_error("null argument"); return LDG_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  auto T0 = std::chrono::steady_clock::now();
  ldg_newton_stats S{};
  const int64_t n = (int64_t)md->N();
  double *G = nullptr, *du = nullptr;
  LDG_TRY(hipMalloc((void**)&G, sizeof(double) * n));
  if (hipMalloc((void**)&du, sizeof(double) * n) != hipSuccess) { hipFree(G); set_error("alloc"); return LDG_ENOMEM; }
  auto cleanup = [&]() { hipFree(G); hipFree(du); };
  ldg_status st = residual_impl(*md, t, u, G, nullptr, false, s);
  double g2 = 0.0;
  if (st == LDG_OK) st = vec_norm2(n, G, md->d_red, &g2, s);
  if (st != LDG_OK) { cleanup(); return st; }
  const double g0 = std::sqrt(g2);
  double gn = g0;
  S.res0 = g0;
  ldg_status result = LDG_OK;
  ldg_gmres_opts lin = opts->lin;
  lin.record_v = lin.record_jz = nullptr;   // recording is a hook of single linear solves
  lin.record_max = 0;
  lin.rtol = opts->eta;
  while (gn > std::max(opts->rtol * g0, opts->atol)) {
    if (S.iters >= opts->maxit) { result = LDG_ENOCONV; set_error("Newton did not converge"); break; }
    if (!std::isfinite(gn)) { result = LDG_EBREAKDOWN; set_error("non-finite Newton residual"); break; }
    if (lin.pc && (opts->bj_refresh == 1 || (opts->bj_refresh == 2 && S.iters == 0))) {
      st = precond_rebuild(lin.pc, t, u, s);
      if (st != LDG_OK) { result = st; break; }
    }
    // J du = -G
    st = vec_axpby(n, -1.0, G, 0.0, G, s);
    if (st == LDG_OK) st = vec_fill(n, 0.0, du, s);
    if (st != LDG_OK) { result = st; break; }
    ldg_gmres_stats gs{};
    st = gmres_impl(*md, t, u, G, du, lin, &gs, s);
    S.gmres_iters += gs.iters;
    S.t_jvp += gs.t_jvp;
    S.t_pc += gs.t_pc;
    S.t_orth += gs.t_orth;
    S.lin_status = st;
    if (st != LDG_OK && st != LDG_ENOCONV) { result = st; break; }
    st = vec_axpby(n, 1.0, du, 1.0, u, s);
    if (st == LDG_OK) st = residual_impl(*md, t, u, G, nullptr, false, s);
    if (st == LDG_OK) st = vec_norm2(n, G, md->d_red, &g2, s);
    if (st != LDG_OK) { result = st; break; }
    gn = std::sqrt(g2);
    ++S.iters;
  }
  S.res_final = gn;
  S.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - T0).count();
  if (stats) *stats = S;
  cleanup();
  return result;
}

}  // extern "C"
