// Block-Jacobi preconditioner: exact element diagonal blocks of the Jacobian by
// probing (one JVP per element colour and local unknown; elements of one colour
// are at face-graph distance >= 3, beyond the reach of the LDG stencil), batched
// Gauss-Jordan inversion with partial pivoting, and a batched block-matrix
// vector product as the apply (FP64, FP32, or 16-bit storage: bf16 or fp16 with
// a power-of-two scale per row and FP64 accumulation).
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "ldg_internal.hpp"

struct ldg_precond_s {
  int kind = 0;           // 0 block-Jacobi, 1 learned (MLP) composite
  void* mlp_data = nullptr;
  ldg::Model* md;
  int per_variable;
  ldg_precision prec;     // storage precision of the inverse blocks
  int nb;                 // block size
  int64_t nblocks;        // E (full) or E * ncu (per variable)
  void* inv = nullptr;    // FP64/FP32: [nblocks][nb][nb], transposed: inv[b][j][i] = (B_b^-1)[i][j]
                          // 16-bit: [nblocks][ng][nb][4], inv[b][g][i][k] = (B_b^-1)[i][4g+k] / scale[b][i]
                          // (zero for 4g+k >= nb)
  float* scale = nullptr; // 16-bit: [nblocks][nb] power-of-two row scales
  int ng = 0;             // 16-bit: column groups of four, ceil(nb / 4)
  double* scratch = nullptr;  // assembled blocks [nblocks][nb][nb] row-major (column-major when colmajor)
  bool colmajor = false;
  int* info = nullptr;        // singular-block counter (device)
  double a0 = 0.0;
};

namespace ldg {

__global__ void k_probe_set(int n, const int32_t* __restrict__ list, int NB, int j, double val,
                            double* __restrict__ v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) v[(int64_t)list[t] * NB + j] = val;
}

// batched seeds: seed column j0 + y of every listed element in the y-th vector
__global__ void k_probe_set_b(int n, const int32_t* __restrict__ list, int NB, int j0, int64_t stride, double val,
                              double* __restrict__ v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) v[blockIdx.y * stride + (int64_t)list[t] * NB + j0 + blockIdx.y] = val;
}

// column j of every listed element's block from Jv
__global__ void k_probe_gather(int n, const int32_t* __restrict__ list, int NB, int nn, int j, int per_variable,
                               const double* __restrict__ Jv, double* __restrict__ blocks) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (per_variable) {
    if (t >= (int64_t)n * nn) return;
    const int64_t K = list[t / nn];
    const int i = t % nn;
    const int cv = j / nn, jn = j % nn;
    const int ncu = NB / nn;
    blocks[(((K * ncu + cv) * nn) + i) * nn + jn] = Jv[K * NB + cv * nn + i];
  } else {
    if (t >= (int64_t)n * NB) return;
    const int64_t K = list[t / NB];
    const int i = t % NB;
    blocks[(K * NB + i) * NB + j] = Jv[K * NB + i];
  }
}

// batched gather: column j0 + y from the y-th result vector
// (colmajor: each block stored column-major, block[j][i], so that one column is
// one contiguous write)
__global__ void k_probe_gather_b(int n, const int32_t* __restrict__ list, int NB, int nn, int j0, int64_t stride,
                                 int per_variable, int colmajor, const double* __restrict__ Jv,
                                 double* __restrict__ blocks) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = j0 + blockIdx.y;
  Jv += blockIdx.y * stride;
  if (per_variable) {
    if (t >= (int64_t)n * nn) return;
    const int64_t K = list[t / nn];
    const int i = t % nn;
    const int cv = j / nn, jn = j % nn;
    const int ncu = NB / nn;
    const int64_t o = ((K * ncu + cv) * nn) * nn;
    blocks[o + (colmajor ? (int64_t)jn * nn + i : (int64_t)i * nn + jn)] = Jv[K * NB + cv * nn + i];
  } else {
    if (t >= (int64_t)n * NB) return;
    const int64_t K = list[t / NB];
    const int i = t % NB;
    blocks[K * NB * NB + (colmajor ? (int64_t)j * NB + i : (int64_t)i * NB + j)] = Jv[K * NB + i];
  }
}

// 16-bit codes: bf16 by round-to-nearest-even of the FP32 value; fp16 by the
// hardware conversion
__device__ inline uint16_t to_bf16(double x) {
  uint32_t u = __float_as_uint((float)x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline uint16_t to_fp16(double x) {
  const _Float16 h = (_Float16)(float)x;
  return __builtin_bit_cast(uint16_t, h);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ inline double from_bf16(uint32_t c) { return (double)__uint_as_float(c << 16); }
__device__ inline double from_fp16(uint32_t c) { return (double)(float)__builtin_bit_cast(_Float16, (uint16_t)c); }

// In-place Gauss-Jordan inversion with row pivoting of one nb x nb block per
// work-group (A in LDS when it fits, otherwise in global memory), written out
// transposed in the storage precision.  H = 0: S-typed entries; H = 1 (bf16) or
// 2 (fp16): the grouped 16-bit layout with row scales.
template <class S, int H>
__global__ void __launch_bounds__(256) k_gj_invert(int nb, double* __restrict__ blocks, S* __restrict__ inv,
                                                   float* __restrict__ scale, int use_lds, int* __restrict__ info) {
  extern __shared__ double lds[];
  __shared__ int piv[128];
  __shared__ double fcol[128];
  __shared__ int pidx;
  __shared__ double bestv, pval;
  const int64_t b = blockIdx.x;
  double* G = blocks + b * (int64_t)nb * nb;
  double* A = use_lds ? lds : G;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nn2 = nb * nb;
  const int rpp = nt / nb;                 // rows per pass of the update (nb <= 128 < nt)
  const int jc = tid % nb, r0 = tid / nb;
  if (use_lds)
    for (int t = tid; t < nn2; t += nt) A[t] = G[t];
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    if (tid < 64) {
      double bv = -1.0;
      int bi = k;
      for (int i = k + tid; i < nb; i += 64) {
        const double a = fabs(A[i * nb + k]);
        if (a > bv) { bv = a; bi = i; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_down(bv, off, 64);
        const int oi = __shfl_down(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if (tid == 0) { pidx = bi; bestv = bv; piv[k] = bi; pval = A[bi * nb + k]; }
    }
    __syncthreads();
    const int p = pidx;
    const double pv = pval;
    const double ipv = pv != 0.0 ? 1.0 / pv : 0.0;
    if (tid == 0 && !(bestv > 0.0)) atomicAdd(info, 1);
    // interchange rows k and p and scale the new row k, in every column but k;
    // fcol = the new column k off row k.  Column k itself is only read here: the
    // update below writes all of it (the inverse's column k is -fcol / pv off
    // the diagonal and 1 / pv on it)
    for (int j = tid; j < nb; j += nt) {
      if (j != k) {
        const double akj = A[k * nb + j], apj = A[p * nb + j];
        A[k * nb + j] = apj * ipv;
        if (p != k) A[p * nb + j] = akj;
      }
      fcol[j] = (j == k) ? 0.0 : A[(j == p ? k : j) * nb + k];
    }
    __syncthreads();
    // rank-1 update of the other rows: thread (r0, j) owns column j of rows r0, r0 + rpp, ...
    // (four rows per round, all loads issued before the stores: every entry is
    // read and written by its own thread only, so the reordering is exact)
    if (tid == 0) A[k * nb + k] = ipv;
    if (r0 < rpp) {
      const bool kcol = jc == k;
      const double akj = kcol ? ipv : A[k * nb + jc];
      int i = r0;
      for (; i + 3 * rpp < nb; i += 4 * rpp) {
        double a[4], f[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          a[t] = A[(i + t * rpp) * nb + jc];
          f[t] = fcol[i + t * rpp];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (i + t * rpp != k) A[(i + t * rpp) * nb + jc] = (kcol ? 0.0 : a[t]) - f[t] * akj;
      }
      for (; i < nb; i += rpp) {
        if (i == k) continue;
        const double base = kcol ? 0.0 : A[i * nb + jc];
        A[i * nb + jc] = base - fcol[i] * akj;
      }
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, in reverse order
  for (int k = nb - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k)
      for (int i = tid; i < nb; i += nt) {
        const double t = A[i * nb + k];
        A[i * nb + k] = A[i * nb + p];
        A[i * nb + p] = t;
      }
    __syncthreads();
  }
  if constexpr (H == 0) {
    S* out = inv + b * (int64_t)nb * nb;
    if (r0 < rpp)
      for (int j = r0; j < nb; j += rpp) out[j * nb + jc] = (S)A[jc * nb + j];   // out[j][i] = A[i][j]
  } else {
    // row i scaled by the power of two 2^e >= max_j |A[i][j]| (exact), so every code is in (-1, 1)
    const int ng = (nb + 3) / 4;
    for (int i = tid; i < nb; i += nt) {
      double mx = 0.0;
      for (int j = 0; j < nb; ++j) mx = fmax(mx, fabs(A[i * nb + j]));
      int e = 0;
      if (mx > 0.0) (void)frexp(mx, &e);
      fcol[i] = ldexp(1.0, -e);
      scale[b * nb + i] = (float)ldexp(1.0, e);
    }
    __syncthreads();
    S* out = inv + b * (int64_t)ng * nb * 4;
    for (int t = tid; t < ng * nb * 4; t += nt) {
      const int g = t / (nb * 4), i = (t / 4) % nb, j = 4 * g + (t & 3);
      const double a = j < nb ? A[i * nb + j] * fcol[i] : 0.0;
      out[t] = H == 1 ? to_bf16(a) : to_fp16(a);
    }
  }
}

// one double from a lane given by a wave-uniform index
__device__ inline double lane_bcast(double v, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffu), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Gauss-Jordan inversion of 64 x 64 blocks, one wave per block, lane r holding
// row r in registers.  Row pivoting without interchanges: the pivot of column k
// is the unused row of largest magnitude (lowest row on ties), broadcast to the
// wave through LDS.  The in-place update leaves X with inverse[k][l] =
// X[piv[k]][m] where piv[m] = l, so lane r, the pivot of step k_r, writes its row
// as row k_r of the inverse, entry m to column piv[m].  Output layouts and the
// singular-block count as k_gj_invert.
template <class S, int H>
__global__ void __launch_bounds__(64) k_gj_invert64(const double* __restrict__ blocks, S* __restrict__ inv,
                                                    float* __restrict__ scale, int colmajor,
                                                    int* __restrict__ info) {
  constexpr int NB = 64;
  __shared__ int piv[NB];
  __shared__ double rowp[NB];   // the pivot row, broadcast through LDS
  const int r = threadIdx.x;
  const int64_t b = blockIdx.x;
  double x[NB];
  if (colmajor) {   // entry (r, j) at j * NB + r: consecutive lanes read consecutive words
    const double* g = blocks + b * (NB * NB) + r;
#pragma unroll
    for (int j = 0; j < NB; ++j) x[j] = g[j * NB];
  } else {
    const double* g = blocks + b * (NB * NB) + (int64_t)r * NB;
#pragma unroll
    for (int j = 0; j < NB; j += 2) {
      const double2 t = *reinterpret_cast<const double2*>(g + j);
      x[j] = t.x;
      x[j + 1] = t.y;
    }
  }
  bool used = false, singular = false;
  int myk = 0;
  // the pivot loop runs at run time; the entries stay in registers because every
  // access to x is in a fully unrolled column loop (column k picked by selects)
  for (int k = 0; k < NB; ++k) {
    double xk = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) xk = (j == k) ? x[j] : xk;
    double bv = used ? -1.0 : fabs(xk);
    int bi = r;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    const int p = __builtin_amdgcn_readfirstlane(bi);
    const double pv = lane_bcast(xk, p);
    if (!(bv > 0.0)) singular = true;
    const double ipv = pv != 0.0 ? 1.0 / pv : 0.0;
    const bool me = r == p;
    if (me) {
      used = true;
      myk = k;
    }
    if (r == 0) piv[k] = p;
    const double f = me ? 0.0 : xk;
    const double nk = me ? ipv : -f * ipv;
    if (me) {
#pragma unroll
      for (int j = 0; j < NB; ++j) rowp[j] = x[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const double pj = rowp[j] * ipv;
      const double nv = me ? pj : x[j] - f * pj;
      x[j] = (j == k) ? nk : nv;
    }
    __syncthreads();
  }
  __syncthreads();
  if (r == 0 && singular) atomicAdd(info, 1);
  if constexpr (H == 0) {
    S* out = inv + b * (NB * NB);
#pragma unroll
    for (int m = 0; m < NB; ++m) out[piv[m] * NB + myk] = (S)x[m];   // out[j][i] = inverse[i][j]
  } else {
    double mx = 0.0;
#pragma unroll
    for (int m = 0; m < NB; ++m) mx = fmax(mx, fabs(x[m]));
    int e = 0;
    if (mx > 0.0) (void)frexp(mx, &e);
    const double sc = ldexp(1.0, -e);
    scale[b * NB + myk] = (float)ldexp(1.0, e);
    S* out = inv + b * (NB * NB);
#pragma unroll
    for (int m = 0; m < NB; ++m) {
      const int j = piv[m];
      const double a = x[m] * sc;
      out[((j >> 2) * NB + myk) * 4 + (j & 3)] = H == 1 ? to_bf16(a) : to_fp16(a);
    }
  }
}

// z_b = B_b^-1 r_b with the transposed inverse (M[j][i] = inverse[i][j]): one
// thread per row, bpb blocks per work-group, r_b staged in LDS.  For each j the
// threads of a block read one contiguous row of M; four partial sums keep four
// loads in flight per thread.  The inverses are streamed once per apply (far
// larger than the caches): with nb = 64 every row of M fills whole cache lines
// and is read with nontemporal loads; for other sizes consecutive rows share
// lines, which plain loads reuse (nontemporal ones measured slower there).
// NB > 0: block size fixed at compile time (loop fully unrolled); NB = 0: any
// block size.
// O: storage type of z (double; float for the FP32-state solvers)
template <class S, int NB, class O = double>
__global__ void __launch_bounds__(1024) k_bj_apply(int nb_rt, int64_t nblocks, int bpb, const S* __restrict__ inv,
                                                  const double* __restrict__ r, O* __restrict__ z) {
  extern __shared__ double rs[];
  const int nb = NB > 0 ? NB : nb_rt;
  const int lb = threadIdx.x / nb, i = threadIdx.x % nb;
  const int64_t b = (int64_t)blockIdx.x * bpb + lb;
  const bool act = lb < bpb && b < nblocks;
  if (act) rs[lb * nb + i] = r[b * nb + i];
  __syncthreads();
  if (!act) return;
  const S* M = inv + b * (int64_t)nb * nb + i;
  const double* rb = rs + lb * nb;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (NB > 0) {
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j & 3] += (double)__builtin_nontemporal_load(M + j * NB) * rb[j];
  } else {
    int j = 0;
    for (; j + 4 <= nb; j += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += (double)M[(j + u) * nb] * rb[j + u];
    }
    for (; j < nb; ++j) acc[0] += (double)M[j * nb] * rb[j];
  }
  z[b * nb + i] = (O)((acc[0] + acc[1]) + (acc[2] + acc[3]));
}

// z_b = B_b^-1 r_b from the 16-bit grouped layout: one thread per row, one
// 8-byte load per group of four columns (a wave reads 512 contiguous bytes),
// decoded and accumulated in FP64, times the row scale.  H = 1 bf16, 2 fp16.
template <int H>
__device__ inline void decode4(u32x2 w, double* e) {
  if constexpr (H == 1) {
    e[0] = from_bf16(w.x & 0xffffu); e[1] = from_bf16(w.x >> 16); e[2] = from_bf16(w.y & 0xffffu); e[3] = from_bf16(w.y >> 16);
  } else {
    e[0] = from_fp16(w.x & 0xffffu); e[1] = from_fp16(w.x >> 16); e[2] = from_fp16(w.y & 0xffffu); e[3] = from_fp16(w.y >> 16);
  }
}

template <int H, int NG, class O = double>
__global__ void __launch_bounds__(1024) k_bj_apply16(int nb, int ng_rt, int64_t nblocks, int bpb,
                                                    const uint16_t* __restrict__ inv, const float* __restrict__ scale,
                                                    const double* __restrict__ r, O* __restrict__ z) {
  extern __shared__ double rs[];
  const int ng = NG > 0 ? NG : ng_rt;
  const int lb = threadIdx.x / nb, i = threadIdx.x % nb;
  const int64_t b = (int64_t)blockIdx.x * bpb + lb;
  const bool act = lb < bpb && b < nblocks;
  const u32x2* M = reinterpret_cast<const u32x2*>(inv + (act ? b : 0) * (int64_t)ng * nb * 4) + i;
  u32x2 w[NG > 0 ? NG : 1];
  if constexpr (NG > 0) {
    // group count fixed at compile time: the (at most two per thread) entries
    // of r are requested first, then the whole row of codes, so that waiting
    // for r (the oldest loads) does not wait for the codes.  Loads use clamped
    // in-bounds indices (threads past the last block read block 0's codes,
    // unused); padding entries are zeroed by the selects.
    const int tot = bpb * NG * 4;
    double rv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = threadIdx.x + h * blockDim.x;
      const int l = t / (NG * 4), j = t % (NG * 4);
      const int64_t bb = (int64_t)blockIdx.x * bpb + l;
      const bool ok = t < tot && j < nb && bb < nblocks;
      const double x = r[(ok ? bb : 0) * nb + (ok ? j : 0)];
      rv[h] = ok ? x : 0.0;
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) w[g] = __builtin_nontemporal_load(M + g * nb);
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (threadIdx.x + h * blockDim.x < tot) rs[threadIdx.x + h * blockDim.x] = rv[h];
  } else {
    // r_b staged with zeros up to 4 ng
    for (int t = threadIdx.x; t < bpb * ng * 4; t += blockDim.x) {
      const int l = t / (ng * 4), j = t % (ng * 4);
      const int64_t bb = (int64_t)blockIdx.x * bpb + l;
      rs[t] = (j < nb && bb < nblocks) ? r[bb * nb + j] : 0.0;
    }
  }
  __syncthreads();
  if (!act) return;
  const double* rb = rs + lb * ng * 4;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  auto group = [&](int g, u32x2 wg) {
    double e[4];
    decode4<H>(wg, e);
    double t = acc[g & 3];
#pragma unroll
    for (int k = 0; k < 4; ++k) t = fma(e[k], rb[4 * g + k], t);
    acc[g & 3] = t;
  };
  if constexpr (NG > 0) {
#pragma unroll
    for (int g = 0; g < NG; ++g) group(g, w[g]);
  } else {
#pragma unroll 4
    for (int g = 0; g < ng; ++g) group(g, __builtin_nontemporal_load(M + (int64_t)g * nb));
  }
  z[b * nb + i] = (O)((double)scale[b * nb + i] * ((acc[0] + acc[1]) + (acc[2] + acc[3])));
}

static bool is16(ldg_precision p) { return p == LDG_BF16 || p == LDG_FP16; }

// probe = LDG_FP32 for blocks that are stored in FP32 anyway (the probing JVPs
// then run in FP32 too)
// colmajor: blocks stored column-major (the block-Jacobi build of 64 x 64 blocks,
// whose one-wave inversion then reads each row with coalesced loads); only the
// library's own models take it
static ldg_status assemble_blocks(Model& md, const ldg_time* t, const double* u_lin, int per_variable,
                                  double* blocks, ldg_precision probe, hipStream_t s, bool colmajor = false) {
  Mesh& m = *md.mesh;
  const int NB = md.ncu * m.nn;
  const int64_t n = (int64_t)md.N();
  ldg_status st;
  if (!md.linear && md.hasq) {
    md.q_of[1] = nullptr;
    st = form_q_cache64(md, u_lin, s);
    if (st != LDG_OK) return st;
    if (probe == LDG_FP32) {
      st = form_q_cache32(md, u_lin, PM_FP32, s);
      if (st != LDG_OK) return st;
    }
  }
  // the probing JVPs run on element subsets: rows on the seeded colour only,
  // the q tangent on the colour and its face neighbours (the other entries of
  // Jv and of the q tangent are left stale and never read)
  struct SubsetReset {
    Mesh& m;
    ~SubsetReset() {
      m.sub_list[0] = m.sub_list[1] = nullptr;
      m.sub_count[0] = m.sub_count[1] = 0;
      m.batch = 1;
      m.bsn = m.bsq = 0;
      m.probe_nbr = false;
    }
  } reset{m};
  if (md.kind != LDG_MODEL_USER) {
    // B seed columns per launch (blockIdx.y), so that one colour's products fill
    // the GPU: about 4096 elements per launch, at most 16 products, and at most
    // 1 GiB of probing vectors (direction, result, tangent of q per product)
    int64_t maxcnt = 1;
    for (int c = 0; c < m.ncolors; ++c) maxcnt = std::max<int64_t>(maxcnt, m.nbhd_off[c + 1] - m.nbhd_off[c]);
    const int64_t nq = md.hasq ? (int64_t)m.E * md.ncu * m.nd * m.nn : 0;
    const int64_t per = 2 * n + nq;   // doubles per product (the FP32 tangent of q uses half of its share)
    int B = (int)std::min<int64_t>(16, std::max<int64_t>(1, 4096 / maxcnt));
    B = (int)std::min<int64_t>(B, std::max<int64_t>(1, (int64_t(1) << 27) / per));
    B = std::min(B, NB);
    if (md.probe_batch < B) {
      hipFree(md.d_probe);
      md.d_probe = nullptr;
      md.probe_batch = 0;
      if (hipMalloc((void**)&md.d_probe, sizeof(double) * per * B) != hipSuccess) {
        (void)hipGetLastError();
        set_error("block probing: out of device memory for the batched probing vectors");
        return LDG_ENOMEM;
      }
      md.probe_batch = B;
    }
    double* vb = md.d_probe;
    double* Jvb = vb + n * B;
    void* dqb = Jvb + n * B;
    const bool fp32 = probe == LDG_FP32;
    const TimeDev td = make_time(t, false);
    void* qc = fp32 ? (void*)md.d_q32 : (void*)md.d_q;
    if ((st = vec_fill(n * B, 0.0, vb, s)) != LDG_OK) return st;
    m.bsn = n;
    m.bsq = nq;
    // Navier-Stokes on an affine mesh with distinct face neighbours and the
    // linearization point's traces formed: the tangent kernel forms the
    // neighbours' tangent-of-q traces in closed form, so the tangent of q is
    // needed on the seeded colour only
    m.probe_nbr = md.kind == LDG_MODEL_NS && m.affine && m.nbr_distinct &&
                  (fp32 ? (md.d_tr32 && md.tr32_valid) : (md.d_tr && md.tr_of == u_lin));
    for (int c = 0; c < m.ncolors; ++c) {
      const int cnt = (int)(m.color_off[c + 1] - m.color_off[c]);
      const int32_t* list = m.d_color_list + m.color_off[c];
      m.sub_list[0] = m.probe_nbr ? list : m.d_color_nbhd + m.nbhd_off[c];
      m.sub_count[0] = m.probe_nbr ? cnt : m.nbhd_off[c + 1] - m.nbhd_off[c];
      m.sub_list[1] = list;
      m.sub_count[1] = cnt;
      for (int j0 = 0; j0 < NB; j0 += B) {
        const int b = std::min(B, NB - j0);
        m.batch = b;
        hipLaunchKernelGGL(k_probe_set_b, dim3((cnt + 255) / 256, b), dim3(256), 0, s, cnt, list, NB, j0, n, 1.0, vb);
        if (md.linear) {
          if ((st = op_grad(md, vb, dqb, fp32, false, s)) != LDG_OK) return st;
          if ((st = op_resid(md, td, vb, dqb, Jvb, fp32, false, s)) != LDG_OK) return st;
        } else {
          if (md.hasq && (st = op_grad(md, vb, dqb, fp32, false, s)) != LDG_OK) return st;
          if ((st = op_jvp_nonlinear(md, td, u_lin, qc, vb, dqb, Jvb, fp32, s)) != LDG_OK)
            return st;
        }
        const int64_t tot = per_variable ? (int64_t)cnt * m.nn : (int64_t)cnt * NB;
        hipLaunchKernelGGL(k_probe_gather_b, dim3((unsigned)((tot + 255) / 256), b), dim3(256), 0, s, cnt, list, NB,
                           m.nn, j0, n, per_variable, colmajor ? 1 : 0, Jvb, blocks);
        hipLaunchKernelGGL(k_probe_set_b, dim3((cnt + 255) / 256, b), dim3(256), 0, s, cnt, list, NB, j0, n, 0.0, vb);
      }
    }
    LDG_TRY(hipGetLastError());
    return LDG_OK;
  }
  double* v = md.d_tmp;
  double* Jv = md.d_tmp2;
  st = vec_fill(n, 0.0, v, s);
  if (st != LDG_OK) return st;
  for (int c = 0; c < m.ncolors; ++c) {
    const int cnt = (int)(m.color_off[c + 1] - m.color_off[c]);
    const int32_t* list = m.d_color_list + m.color_off[c];
    m.sub_list[0] = m.d_color_nbhd + m.nbhd_off[c];
    m.sub_count[0] = m.nbhd_off[c + 1] - m.nbhd_off[c];
    m.sub_list[1] = list;
    m.sub_count[1] = cnt;
    for (int j = 0; j < NB; ++j) {
      hipLaunchKernelGGL(k_probe_set, dim3((cnt + 255) / 256), dim3(256), 0, s, cnt, list, NB, j, 1.0, v);
      st = jvp_impl(md, t, u_lin, v, Jv, probe, true, s);
      if (st != LDG_OK) return st;
      const int64_t tot = per_variable ? (int64_t)cnt * m.nn : (int64_t)cnt * NB;
      hipLaunchKernelGGL(k_probe_gather, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, cnt, list, NB, m.nn, j,
                         per_variable, Jv, blocks);
      hipLaunchKernelGGL(k_probe_set, dim3((cnt + 255) / 256), dim3(256), 0, s, cnt, list, NB, j, 0.0, v);
    }
  }
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

static ldg_status invert_blocks(ldg_precond_s* pc, hipStream_t s) {
  const int nb = pc->nb;
  const size_t bytes = (size_t)nb * nb * sizeof(double);
  // the block in LDS when it fits beside the kernel's ~1.6 KB of static LDS
  static int lds_limit = -1;
  if (lds_limit < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 64 * 1024;
    lds_limit = v;
    (void)hipGetLastError();
  }
  const int use_lds = bytes + 2048 <= (size_t)lds_limit ? 1 : 0;
  if (use_lds && bytes > 48 * 1024) {
    const void* f = pc->prec == LDG_FP32   ? (const void*)k_gj_invert<float, 0>
                    : pc->prec == LDG_BF16 ? (const void*)k_gj_invert<uint16_t, 1>
                    : pc->prec == LDG_FP16 ? (const void*)k_gj_invert<uint16_t, 2>
                                           : (const void*)k_gj_invert<double, 0>;
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipGetLastError();
  }
  if (nb > 128) { set_error("block size above 128"); return LDG_EUNSUPPORTED; }
  if (zero_int(pc->info, s) != LDG_OK) return LDG_EDEVICE;
  if (nb == 64) {
    // one wave per block, the block in registers
    const dim3 g64((unsigned)pc->nblocks);
    if (pc->prec == LDG_FP32)
      hipLaunchKernelGGL((k_gj_invert64<float, 0>), g64, dim3(64), 0, s, pc->scratch, (float*)pc->inv, pc->scale,
                         (int)pc->colmajor, pc->info);
    else if (pc->prec == LDG_BF16)
      hipLaunchKernelGGL((k_gj_invert64<uint16_t, 1>), g64, dim3(64), 0, s, pc->scratch, (uint16_t*)pc->inv,
                         pc->scale, (int)pc->colmajor, pc->info);
    else if (pc->prec == LDG_FP16)
      hipLaunchKernelGGL((k_gj_invert64<uint16_t, 2>), g64, dim3(64), 0, s, pc->scratch, (uint16_t*)pc->inv,
                         pc->scale, (int)pc->colmajor, pc->info);
    else
      hipLaunchKernelGGL((k_gj_invert64<double, 0>), g64, dim3(64), 0, s, pc->scratch, (double*)pc->inv, pc->scale,
                         (int)pc->colmajor, pc->info);
  } else {
  const int threads = 256;
  const size_t lds = use_lds ? bytes : 0;
  const dim3 grid((unsigned)pc->nblocks);
  if (pc->prec == LDG_FP32)
    hipLaunchKernelGGL((k_gj_invert<float, 0>), grid, dim3(threads), lds, s, nb, pc->scratch, (float*)pc->inv,
                       pc->scale, use_lds, pc->info);
  else if (pc->prec == LDG_BF16)
    hipLaunchKernelGGL((k_gj_invert<uint16_t, 1>), grid, dim3(threads), lds, s, nb, pc->scratch, (uint16_t*)pc->inv,
                       pc->scale, use_lds, pc->info);
  else if (pc->prec == LDG_FP16)
    hipLaunchKernelGGL((k_gj_invert<uint16_t, 2>), grid, dim3(threads), lds, s, nb, pc->scratch, (uint16_t*)pc->inv,
                       pc->scale, use_lds, pc->info);
  else
    hipLaunchKernelGGL((k_gj_invert<double, 0>), grid, dim3(threads), lds, s, nb, pc->scratch, (double*)pc->inv,
                       pc->scale, use_lds, pc->info);
  }
  LDG_TRY(hipGetLastError());
  int h_info = 0;
  LDG_TRY(hipMemcpyAsync(&h_info, pc->info, sizeof(int), hipMemcpyDeviceToHost, s));
  LDG_TRY(hipStreamSynchronize(s));
  if (h_info != 0) { set_error("singular Jacobian block"); return LDG_EBREAKDOWN; }
  return LDG_OK;
}

ldg_status precond_rebuild(ldg_precond_s* pc, const ldg_time* t, const double* u_lin, hipStream_t s) {
  if (pc->kind == 1) {
    set_error("the learned preconditioner is rebuilt through its block-Jacobi part");
    return LDG_EINVAL;
  }
  // 64 x 64 blocks of the library's own models: column-major for k_gj_invert64
  pc->colmajor = pc->nb == 64 && pc->md->kind != LDG_MODEL_USER;
  ldg_status st = assemble_blocks(*pc->md, t, u_lin, pc->per_variable, pc->scratch,
                                  pc->prec == LDG_FP64 ? LDG_FP64 : LDG_FP32, s, pc->colmajor);
  if (st != LDG_OK) return st;
  return invert_blocks(pc, s);
}

ldg_status mlp_precond_apply(void* data, const double* r, double* z, hipStream_t s);
void* mlp_precond_create(Model* md, struct MlpNet* net, ldg_precond_s* bj, int composite, ldg_status* status);
void mlp_dims(const struct MlpNet* net, int* in_dim, int* out_dim);
void mlp_precond_destroy(void* data);

template <class O>
static ldg_status bj_apply(ldg_precond_s* pc, const double* r, O* z, hipStream_t s) {
  const int nb = pc->nb;
  int bpb = 256 / nb;
  if (bpb < 1) bpb = 1;
  const unsigned grid = (unsigned)((pc->nblocks + bpb - 1) / bpb);
  const size_t sh = (size_t)bpb * nb * sizeof(double);
  const dim3 thr(bpb * nb);
  if (nb > 1024) { set_error("block-Jacobi blocks larger than 1024 rows"); return LDG_EUNSUPPORTED; }
  if (is16(pc->prec)) {
    const size_t sh16 = (size_t)bpb * pc->ng * 4 * sizeof(double);
    const uint16_t* inv = (const uint16_t*)pc->inv;
    // compile-time group counts for the common block sizes: 16 (nb 64), 25
    // (nb 100), 7 (nb 25, 27), 4 (nb 16)
#define LDG_APPLY16(HH, NGC)                                                                                         \
  hipLaunchKernelGGL((k_bj_apply16<HH, NGC, O>), dim3(grid), thr, sh16, s, nb, pc->ng, pc->nblocks, bpb, inv, pc->scale, \
                     r, z)
#define LDG_APPLY16_ALL(HH)                     \
  switch (pc->ng) {                             \
    case 16: LDG_APPLY16(HH, 16); break;        \
    case 25: LDG_APPLY16(HH, 25); break;        \
    case 7: LDG_APPLY16(HH, 7); break;          \
    case 4: LDG_APPLY16(HH, 4); break;          \
    default: LDG_APPLY16(HH, 0); break;         \
  }
    if (pc->prec == LDG_BF16) {
      LDG_APPLY16_ALL(1)
    } else {
      LDG_APPLY16_ALL(2)
    }
#undef LDG_APPLY16_ALL
#undef LDG_APPLY16
  } else if (pc->prec == LDG_FP32) {
    if (nb == 64)
      hipLaunchKernelGGL((k_bj_apply<float, 64, O>), dim3(grid), thr, sh, s, nb, pc->nblocks, bpb, (const float*)pc->inv, r, z);
    else
      hipLaunchKernelGGL((k_bj_apply<float, 0, O>), dim3(grid), thr, sh, s, nb, pc->nblocks, bpb, (const float*)pc->inv, r, z);
  } else {
    if (nb == 64)
      hipLaunchKernelGGL((k_bj_apply<double, 64, O>), dim3(grid), thr, sh, s, nb, pc->nblocks, bpb, (const double*)pc->inv, r, z);
    else
      hipLaunchKernelGGL((k_bj_apply<double, 0, O>), dim3(grid), thr, sh, s, nb, pc->nblocks, bpb, (const double*)pc->inv, r, z);
  }
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

ldg_status precond_apply_impl(ldg_precond_s* pc, const double* r, double* z, hipStream_t s) {
  if (pc->kind == 1) return mlp_precond_apply(pc->mlp_data, r, z, s);
  return bj_apply<double>(pc, r, z, s);
}

// the block-Jacobi apply with z in FP32 storage (FP32-state solvers)
ldg_status precond_apply_impl32(ldg_precond_s* pc, const double* r, float* z, hipStream_t s) {
  if (pc->kind == 1) {
    set_error("the FP32-state solver takes the block-Jacobi preconditioner, not the learned one");
    return LDG_EUNSUPPORTED;
  }
  return bj_apply<float>(pc, r, z, s);
}

int precond_kind(const ldg_precond_s* pc) { return pc ? pc->kind : -1; }

ldg_status mlp_precond_count_nonfinite(void* data, const double* z, int64_t n, int* host_cnt, hipStream_t s);
ldg_precond_s* mlp_precond_fallback(void* data);

ldg_precond_s* precond_fallback(ldg_precond_s* pc) {
  return (pc && pc->kind == 1) ? mlp_precond_fallback(pc->mlp_data) : nullptr;
}

ldg_status precond_count_nonfinite(ldg_precond_s* pc, const double* z, int64_t n, int* host_cnt, hipStream_t s) {
  if (!pc || pc->kind != 1) { *host_cnt = 0; return LDG_OK; }
  return mlp_precond_count_nonfinite(pc->mlp_data, z, n, host_cnt, s);
}

}  // namespace ldg

using namespace ldg;


extern "C" {

ldg_status ldg_jacobian_blocks(ldg_model md, const ldg_time* t, const double* u_lin, int per_variable, double* blocks,
                               void* stream) {
  LDG_ENTER();
  if (!md || !blocks) { set_error("null argument"); return LDG_EINVAL; }
  if (!md->linear && !u_lin) { set_error("nonlinear model needs u_lin"); return LDG_EINVAL; }
  return assemble_blocks(*md, t, u_lin, per_variable, blocks, LDG_FP64, (hipStream_t)stream);
}

ldg_status ldg_precond_block_jacobi(ldg_model md, const ldg_time* t, const double* u_lin, int per_variable,
                                    ldg_precision factor_prec, void* stream, ldg_precond* out) {
  LDG_ENTER();
  if (!md || !out) { set_error("null argument"); return LDG_EINVAL; }
  if (factor_prec != LDG_FP64 && factor_prec != LDG_FP32 && !is16(factor_prec)) {
    set_error("factor precision must be FP64, FP32, BF16 or FP16");
    return LDG_EINVAL;
  }
  if (!md->linear && !u_lin) { set_error("nonlinear model needs u_lin"); return LDG_EINVAL; }
  auto* pc = new ldg_precond_s();
  pc->md = md;
  pc->per_variable = per_variable ? 1 : 0;
  pc->prec = factor_prec;
  pc->nb = per_variable ? md->mesh->nn : md->ncu * md->mesh->nn;
  pc->nblocks = per_variable ? md->mesh->E * md->ncu : md->mesh->E;
  pc->a0 = t ? t->a0 : 0.0;
  if (pc->nb > 128) { delete pc; set_error("block size above 128"); return LDG_EUNSUPPORTED; }
  const size_t nel = (size_t)pc->nblocks * pc->nb * pc->nb;
  pc->ng = (pc->nb + 3) / 4;
  const size_t inv_bytes = is16(factor_prec) ? (size_t)pc->nblocks * pc->ng * 4 * pc->nb * sizeof(uint16_t)
                                             : nel * (factor_prec == LDG_FP32 ? sizeof(float) : sizeof(double));
  hipError_t e = hipMalloc((void**)&pc->scratch, nel * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&pc->inv, inv_bytes);
  if (e == hipSuccess && is16(factor_prec)) e = hipMalloc((void**)&pc->scale, (size_t)pc->nblocks * pc->nb * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&pc->info, sizeof(int));
  if (e != hipSuccess) {
    hipFree(pc->scratch); hipFree(pc->inv); hipFree(pc->scale); hipFree(pc->info);
    delete pc;
    set_error(std::string("block-Jacobi allocation: ") + hipGetErrorString(e));
    return LDG_ENOMEM;
  }
  ldg_status st = precond_rebuild(pc, t, u_lin, (hipStream_t)stream);
  if (st != LDG_OK) {
    hipFree(pc->scratch); hipFree(pc->inv); hipFree(pc->scale); hipFree(pc->info);
    delete pc;
    return st;
  }
  *out = pc;
  return LDG_OK;
}

ldg_status ldg_precond_apply(ldg_precond pc, const double* r, double* z, void* stream) {
  LDG_ENTER();
  if (!pc || !r || !z) { set_error("null argument"); return LDG_EINVAL; }
  return precond_apply_impl(pc, r, z, (hipStream_t)stream);
}

ldg_status ldg_precond_mlp(ldg_model md, ldg_mlp net, ldg_precond fallback_bj, int composite, ldg_precond* out) {
  LDG_ENTER();
  if (!md || !net || !out) { set_error("null argument"); return LDG_EINVAL; }
  if (md->mesh->nd != 2 || md->ncu != 1) { set_error("element patches are defined for 2D scalar models"); return LDG_EUNSUPPORTED; }
  if (fallback_bj && fallback_bj->kind != 0) { set_error("fallback must be a block-Jacobi preconditioner"); return LDG_EINVAL; }
  if (composite < 0 || composite > 2) { set_error("composite must be 0, 1 or 2"); return LDG_EINVAL; }
  if (composite && !fallback_bj) { set_error("composite forms need the block-Jacobi part"); return LDG_EINVAL; }
  {
    int in_dim = 0, out_dim = 0;
    mlp_dims((const MlpNet*)net, &in_dim, &out_dim);
    const int nn = md->mesh->nn;
    const bool ok = composite == 2 ? (in_dim == 15 * nn && out_dim == 5 * nn * nn && nn <= 64)
                                   : (in_dim == 20 * nn && out_dim == nn);
    if (!ok) {
      set_error(composite == 2 ? "linear form: the network maps 15 nn coefficient features to 5 nn^2 outputs"
                               : "the network maps 20 nn patch features to nn outputs");
      return LDG_EINVAL;
    }
  }
  if (composite == 2 && md->naux != 3) { set_error("the linear form needs aux = [kappa, b_x, b_y]"); return LDG_EUNSUPPORTED; }
  auto* pc = new ldg_precond_s();
  pc->kind = 1;
  pc->md = md;
  pc->nb = 0;
  pc->nblocks = 0;
  ldg_status st = LDG_OK;
  pc->mlp_data = mlp_precond_create(md, (MlpNet*)net, fallback_bj, composite, &st);
  if (!pc->mlp_data) { delete pc; return st == LDG_OK ? LDG_ENOMEM : st; }
  *out = pc;
  return LDG_OK;
}

ldg_status ldg_precond_destroy(ldg_precond pc) {
  LDG_ENTER();
  if (!pc) return LDG_OK;
  if (pc->kind == 1) { mlp_precond_destroy(pc->mlp_data); delete pc; return LDG_OK; }
  hipFree(pc->scratch); hipFree(pc->inv); hipFree(pc->scale); hipFree(pc->info);
  delete pc;
  return LDG_OK;
}

}  // extern "C"
