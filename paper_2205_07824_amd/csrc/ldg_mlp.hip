// Element-patch MLP preconditioner: patch gather, GEMMs on MFMA (bf16 operands,
// fp32 accumulation) or FP32 VALU, forward / backward / Adam, and two right
// preconditioners for flexible GMRES, with block-Jacobi as the fallback:
//  * residual form: z = B^-1 r + s N(patch(r) / s), the network evaluated on
//    every preconditioner input;
//  * linear form: z = B^-1 (r + A_K patch(r)), where the network maps the
//    coefficient patch of element K to its patch-to-element matrix A_K once,
//    when the preconditioner is created (a fixed linear operator, as Krylov
//    methods assume), trained with the bilinear loss of
//    ldg_mlp_train_step_bilinear.
//
// Network: y = W3 relu(W2 relu(W1 x + b1) + b2) + b3, weights row-major
// W_l[out][in], FP32 master copies; the GEMM kernel converts operands to bf16
// (round to nearest even) when it stages them into LDS.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "ldg_internal.hpp"

namespace ldg {

struct MlpNet {
  int in_dim, width, out_dim;
  bool bf16 = true;
  int64_t nparams = 0;
  float* params = nullptr;   // packed W1 b1 W2 b2 W3 b3
  float* grads = nullptr;
  float* m1 = nullptr;       // Adam moments
  float* m2 = nullptr;
  int64_t cap = 0;           // batch capacity of the work buffers
  float* H1 = nullptr;       // [cap][width] post-activation
  float* H2 = nullptr;
  float* Yo = nullptr;       // [cap][out]
  float* dY = nullptr;
  float* dH2 = nullptr;      // [cap][width]
  float* dH1 = nullptr;
  float* part = nullptr;     // split-K partials
  int64_t part_cap = 0;
  float* loss_dev = nullptr;
  int64_t t = 0;             // Adam step
  int64_t off[6];            // offsets of W1 b1 W2 b2 W3 b3 in params
};

// ----------------------------------------------------------------- bf16 ---
__device__ inline unsigned short f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// --------------------------------------------------------------- GEMM ------
// C(m,n) = act( sum_k A(m,k) B(k,n) + bias[n] ) with arbitrary strides.
// 64x64 output tile per 256-thread work-group; K in steps of 16.  Split-K:
// blockIdx.z selects a K range and writes partials Cp[z] (reduced afterwards).
// BF16 path: each wave computes a 32x32 sub-tile as 2x2 MFMA 16x16x16 tiles.
// FP32 path: each thread computes a 4x4 micro-tile with FMAs.
constexpr int GT = 64, GK = 16;

template <bool BF16>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, int kchunk, const float* __restrict__ A, int64_t sam,
                                              int64_t sak, const float* __restrict__ B, int64_t sbk, int64_t sbn,
                                              float* __restrict__ C, int64_t scm, int64_t scn, int64_t szc,
                                              const float* __restrict__ bias, int act) {
  __shared__ float As[GT][GK + 1];   // A tile [m][k]
  __shared__ float Bs[GK][GT + 1];   // B tile [k][n]
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int tid = threadIdx.x;
  float acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  f32x4 cm[2][2];
  if constexpr (BF16) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) cm[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  const int wave = tid >> 6, lane = tid & 63;
  for (int k0 = kbeg; k0 < kend; k0 += GK) {
    // stage A (64 x 16) and B (16 x 64); zero padding outside the matrices / K range
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 256;
      const int am = e / GK, ak = e % GK;
      const int gm = m0 + am, gk = k0 + ak;
      As[am][ak] = (gm < M && gk < kend) ? A[(int64_t)gm * sam + (int64_t)gk * sak] : 0.0f;
      const int bk = e / GT, bn = e % GT;
      const int gk2 = k0 + bk, gn = n0 + bn;
      Bs[bk][bn] = (gn < N && gk2 < kend) ? B[(int64_t)gk2 * sbk + (int64_t)gn * sbn] : 0.0f;
    }
    __syncthreads();
    if constexpr (BF16) {
      // wave tile: rows (wave >> 1) * 32, cols (wave & 1) * 32
      const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
      const int li = lane & 15, kg = lane >> 4;
      bf16x4 af[2], bfr[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) af[a][i] = (short)f2bf(As[wr + a * 16 + li][kg * 4 + i]);
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) bfr[b][i] = (short)f2bf(Bs[kg * 4 + i][wc + b * 16 + li]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) cm[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bfr[b], cm[a][b], 0, 0, 0);
    } else {
      const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
#pragma unroll
      for (int kk = 0; kk < GK; ++kk) {
        float av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) { av[i] = As[tr + i][kk]; bv[i] = Bs[kk][tc + i]; }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i * 4 + j] = fmaf(av[i], bv[j], acc[i * 4 + j]);
      }
    }
    __syncthreads();
  }
  float* Cz = C + (int64_t)blockIdx.z * szc;
  const bool final_pass = gridDim.z == 1;
  auto store = [&](int gm, int gn, float val) {
    if (gm >= M || gn >= N) return;
    if (final_pass) {
      if (bias) val += bias[gn];
      if (act == 1) val = val > 0.0f ? val : 0.0f;
    }
    Cz[(int64_t)gm * scm + (int64_t)gn * scn] = val;
  };
  if constexpr (BF16) {
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int li = lane & 15, kg = lane >> 4;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i) store(m0 + wr + a * 16 + kg * 4 + i, n0 + wc + b * 16 + li, cm[a][b][i]);
  } else {
    const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) store(m0 + tr + i, n0 + tc + j, acc[i * 4 + j]);
  }
}

// sum the split-K partials and apply bias / activation
__global__ void k_splitk_reduce(int M, int N, int nz, const float* __restrict__ P, int64_t szc,
                                float* __restrict__ C, int64_t scm, int64_t scn, const float* __restrict__ bias,
                                int act) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)M * N) return;
  const int m = t / N, n = t % N;
  float s = 0.0f;
  for (int z = 0; z < nz; ++z) s += P[(int64_t)z * szc + (int64_t)m * N + n];
  if (bias) s += bias[n];
  if (act == 1) s = s > 0.0f ? s : 0.0f;
  C[(int64_t)m * scm + (int64_t)n * scn] = s;
}

static ldg_status gemm(MlpNet& net, int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B,
                       int64_t sbk, int64_t sbn, float* C, int64_t scm, int64_t scn, const float* bias, int act,
                       hipStream_t s, bool allow_split = true) {
  if (!A || !B || !C || M <= 0 || N <= 0 || K <= 0) { set_error("GEMM operand missing or empty"); return LDG_EINVAL; }
  const int gx = (N + GT - 1) / GT, gy = (M + GT - 1) / GT;
  int nz = 1;
  // split K when the output has few tiles and K is long (weight gradients); the
  // split needs the partial buffer net.part, so callers that may not allocate
  // pass allow_split = false
  while (allow_split && gx * gy * nz < 256 && K / (nz * 2) >= 256) nz *= 2;
  int kchunk = (K + nz - 1) / nz;
  kchunk = (kchunk + GK - 1) / GK * GK;
  nz = (K + kchunk - 1) / kchunk;
  if (nz == 1) {
    if (net.bf16)
      hipLaunchKernelGGL(k_gemm<true>, dim3(gx, gy, 1), dim3(256), 0, s, M, N, K, kchunk, A, sam, sak, B, sbk, sbn, C,
                         scm, scn, (int64_t)0, bias, act);
    else
      hipLaunchKernelGGL(k_gemm<false>, dim3(gx, gy, 1), dim3(256), 0, s, M, N, K, kchunk, A, sam, sak, B, sbk, sbn, C,
                         scm, scn, (int64_t)0, bias, act);
  } else {
    const int64_t szc = (int64_t)M * N;
    if (net.part_cap < szc * nz) {
      LDG_TRY(hipStreamSynchronize(s));   // earlier split-K work may still read the old buffer
      if (net.part) LDG_TRY(hipFree(net.part));
      net.part_cap = szc * nz;
      LDG_TRY(hipMalloc((void**)&net.part, sizeof(float) * net.part_cap));
    }
    if (net.bf16)
      hipLaunchKernelGGL(k_gemm<true>, dim3(gx, gy, nz), dim3(256), 0, s, M, N, K, kchunk, A, sam, sak, B, sbk, sbn,
                         net.part, (int64_t)N, (int64_t)1, szc, (const float*)nullptr, 0);
    else
      hipLaunchKernelGGL(k_gemm<false>, dim3(gx, gy, nz), dim3(256), 0, s, M, N, K, kchunk, A, sam, sak, B, sbk, sbn,
                         net.part, (int64_t)N, (int64_t)1, szc, (const float*)nullptr, 0);
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((szc + 255) / 256)), dim3(256), 0, s, M, N, nz, net.part, szc,
                       C, scm, scn, bias, act);
  }
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

// ------------------------------------------------------- elementwise -------
// dY = 2 (Y - T) / (B * out); loss partial sums
__global__ void k_mse(int64_t n, float scale, const float* __restrict__ Y, const float* __restrict__ T,
                      float* __restrict__ dY, float* __restrict__ loss) {
  __shared__ float sh[4];
  float s = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = 2.0f * d * scale;
    s += d * d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) t += sh[w];
    atomicAdd(loss, t * scale);
  }
}

// dH *= (H > 0)
__global__ void k_relu_mask(int64_t n, const float* __restrict__ H, float* __restrict__ dH) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(H[i] > 0.0f)) dH[i] = 0.0f;
}

// column sums of X [rows][cols] into g (bias gradients)
__global__ void k_colsum(int64_t rows, int cols, const float* __restrict__ X, float* __restrict__ g) {
  const int c = blockIdx.x;
  __shared__ float sh[4];
  float s = 0.0f;
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) s += X[r * cols + c];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) t += sh[w];
    g[c] = t;
  }
}

__global__ void k_adam(int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_zero_f(int64_t n, float* p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

static ldg_status ensure_cap(MlpNet& net, int64_t B, hipStream_t s) {
  if (B <= net.cap) return LDG_OK;
  // earlier work on the stream may still read the old buffers
  LDG_TRY(hipStreamSynchronize(s));
  float* bufs[] = {net.H1, net.H2, net.Yo, net.dY, net.dH2, net.dH1};
  for (float* b : bufs)
    if (b) LDG_TRY(hipFree(b));
  net.cap = B;
  LDG_TRY(hipMalloc((void**)&net.H1, sizeof(float) * B * net.width));
  LDG_TRY(hipMalloc((void**)&net.H2, sizeof(float) * B * net.width));
  LDG_TRY(hipMalloc((void**)&net.Yo, sizeof(float) * B * net.out_dim));
  LDG_TRY(hipMalloc((void**)&net.dY, sizeof(float) * B * net.out_dim));
  LDG_TRY(hipMalloc((void**)&net.dH2, sizeof(float) * B * net.width));
  LDG_TRY(hipMalloc((void**)&net.dH1, sizeof(float) * B * net.width));
  return LDG_OK;
}

// the three layers with the hidden activations in H1, H2 ([B][width] each)
// (X rows ldx floats apart: the network reads the first in_dim of each)
static ldg_status mlp_layers(MlpNet& net, const float* X, int64_t B, float* H1, float* H2, float* Y, hipStream_t s,
                             bool allow_split, int64_t ldx = -1) {
  if (!Y) { set_error("MLP forward without an output buffer"); return LDG_EINVAL; }
  const int I = net.in_dim, W = net.width, O = net.out_dim;
  if (ldx < 0) ldx = I;
  const float* P = net.params;
  ldg_status st;
  if ((st = gemm(net, (int)B, W, I, X, ldx, 1, P + net.off[0], 1, I, H1, W, 1, P + net.off[1], 1, s, allow_split)) != LDG_OK)
    return st;
  if ((st = gemm(net, (int)B, W, W, H1, W, 1, P + net.off[2], 1, W, H2, W, 1, P + net.off[3], 1, s, allow_split)) != LDG_OK)
    return st;
  return gemm(net, (int)B, O, W, H2, W, 1, P + net.off[4], 1, W, Y, O, 1, P + net.off[5], 0, s, allow_split);
}

// forward into net.H1, net.H2, Y (Y may be net.Yo)
static ldg_status mlp_forward(MlpNet& net, const float* X, int64_t B, float* Y, hipStream_t s, int64_t ldx = -1) {
  ldg_status st = ensure_cap(net, B, s);
  if (st != LDG_OK) return st;
  return mlp_layers(net, X, B, net.H1, net.H2, Y, s, true, ldx);
}

// ---- allocation-free forward --------------------------------------------
// The hidden activations of ldg_mlp_forward_noalloc live in this fixed device
// array (32 MiB; each GPU the library runs on holds its own copy until the
// process ends).  Host code must not pass the array's name to a kernel: on the
// host it is a stand-in, not a device address.  The device address is looked
// up once per device and kept in g_scratch_dev.
constexpr int64_t kScratchFloats = int64_t(1) << 23;
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_dev[kMaxDevices] = {};

// device address of the scratch array on the current device
static ldg_status scratch_address(float** out) {
  int dev = -1;
  LDG_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) { set_error("device index out of range"); return LDG_EDEVICE; }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return LDG_EDEVICE;
    }
    g_scratch_dev[dev] = (float*)p;
  }
  *out = g_scratch_dev[dev];
  return LDG_OK;
}

// gradients of the loss into net.grads from its gradient dY with respect to the
// network output (net.dY [B][out]); X rows ldx floats apart
static ldg_status mlp_backward_dy(MlpNet& net, const float* X, int64_t ldx, int64_t B, hipStream_t s) {
  const int I = net.in_dim, W = net.width, O = net.out_dim;
  const float* P = net.params;
  float* G = net.grads;
  ldg_status st;
  // layer 3: gW3 = dY^T H2, gb3 = colsum dY, dH2 = dY W3
  if ((st = gemm(net, O, W, (int)B, net.dY, 1, O, net.H2, W, 1, G + net.off[4], W, 1, nullptr, 0, s)) != LDG_OK) return st;
  hipLaunchKernelGGL(k_colsum, dim3(O), dim3(256), 0, s, B, O, net.dY, G + net.off[5]);
  if ((st = gemm(net, (int)B, W, O, net.dY, O, 1, P + net.off[4], W, 1, net.dH2, W, 1, nullptr, 0, s)) != LDG_OK) return st;
  hipLaunchKernelGGL(k_relu_mask, dim3((unsigned)((B * W + 255) / 256)), dim3(256), 0, s, B * W, net.H2, net.dH2);
  // layer 2
  if ((st = gemm(net, W, W, (int)B, net.dH2, 1, W, net.H1, W, 1, G + net.off[2], W, 1, nullptr, 0, s)) != LDG_OK) return st;
  hipLaunchKernelGGL(k_colsum, dim3(W), dim3(256), 0, s, B, W, net.dH2, G + net.off[3]);
  if ((st = gemm(net, (int)B, W, W, net.dH2, W, 1, P + net.off[2], W, 1, net.dH1, W, 1, nullptr, 0, s)) != LDG_OK) return st;
  hipLaunchKernelGGL(k_relu_mask, dim3((unsigned)((B * W + 255) / 256)), dim3(256), 0, s, B * W, net.H1, net.dH1);
  // layer 1
  if ((st = gemm(net, W, I, (int)B, net.dH1, 1, W, X, ldx, 1, G + net.off[0], I, 1, nullptr, 0, s)) != LDG_OK) return st;
  hipLaunchKernelGGL(k_colsum, dim3(W), dim3(256), 0, s, B, W, net.dH1, G + net.off[1]);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

// gradients of the mean squared error into net.grads; loss into net.loss_dev
static ldg_status mlp_backward(MlpNet& net, const float* X, const float* T, int64_t B, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f, dim3(1), dim3(64), 0, s, (int64_t)1, net.loss_dev);
  const int64_t ny = B * net.out_dim;
  hipLaunchKernelGGL(k_mse, dim3((unsigned)std::min<int64_t>((ny + 255) / 256, 1024)), dim3(256), 0, s, ny,
                     1.0f / (float)ny, net.Yo, T, net.dY, net.loss_dev);
  return mlp_backward_dy(net, X, net.in_dim, B, s);
}

// Bilinear head of the linear form: per sample b the network output Yo[b] is the
// matrix A_b [nn][5 nn] (row-major) and the prediction is y_b = A_b r_b with
// r_b = X[b][0 : 5 nn] (the residual patch / s).  Loss (1 / (B nn)) sum (y - T)^2
// into *loss; its gradient with respect to Yo, dYo[b][i][j] = 2 (y_bi - T_bi) r_bj / (B nn).
// One 64-thread block per sample.
__global__ void k_bilinear_loss(int64_t B, int nn, const float* __restrict__ X, int64_t ldx,
                                const float* __restrict__ Yo, const float* __restrict__ T, float scale,
                                float* __restrict__ dYo, float* __restrict__ loss) {
  const int64_t b = blockIdx.x;
  if (b >= B) return;
  const int nc = 5 * nn;
  extern __shared__ float sh_bl[];   // r [nc], dy [nn]
  float* rb = sh_bl;
  float* dy = sh_bl + nc;
  for (int j = threadIdx.x; j < nc; j += blockDim.x) rb[j] = X[b * ldx + j];
  __syncthreads();
  float part = 0.0f;
  for (int i = threadIdx.x; i < nn; i += blockDim.x) {
    const float* a = Yo + (b * nn + i) * (int64_t)nc;
    float y = 0.0f;
    for (int j = 0; j < nc; ++j) y = fmaf(a[j], rb[j], y);
    const float d = y - T[b * nn + i];
    dy[i] = 2.0f * d * scale;
    part += d * d;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nn * nc; t += blockDim.x) dYo[b * nn * (int64_t)nc + t] = dy[t / nc] * rb[t % nc];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
  if (threadIdx.x == 0) atomicAdd(loss, part * scale);
}

// ------------------------------------------------------------- patches -----
// Coefficient features of patch slot t / nn, node t % nn (element el, -1 outside
// the domain: zeros), written into the row C = [log kappa (5 nn) | per slot
// b_x / 100 (nn), b_y / 100 (nn)] (velocity scaled by the workload's |b| <= 100).
__device__ inline void patch_coefs(float* C, int t, int64_t el, int nn, const double* __restrict__ aux, int naux) {
  const int npatch = 5 * nn, j = t % nn;
  float lk = 0.f, bx = 0.f, by = 0.f;
  if (el >= 0 && naux >= 3) {
    lk = (float)log(aux[(el * naux + 0) * nn + j]);
    bx = (float)(0.01 * aux[(el * naux + 1) * nn + j]);
    by = (float)(0.01 * aux[(el * naux + 2) * nn + j]);
  }
  C[t] = lk;
  C[npatch + (t / nn) * 2 * nn + j] = bx;
  C[npatch + (t / nn) * 2 * nn + nn + j] = by;
}

// the coefficient features of every element (rows of 15 nn floats)
__global__ void k_coef_patches(int64_t E, int nn, const int32_t* __restrict__ nbr, const double* __restrict__ aux,
                               int naux, float* __restrict__ C) {
  const int64_t K = blockIdx.x;
  if (K >= E) return;
  for (int t = threadIdx.x; t < 5 * nn; t += blockDim.x) {
    const int slot = t / nn;
    const int64_t el = slot == 0 ? K : (int64_t)nbr[K * 4 + (slot - 1)];
    patch_coefs(C + K * 15 * nn, t, el >= 0 ? el : -1, nn, aux, naux);
  }
}

// y_K = r_K + A_K patch(r)_K: A [E][nn][5 nn] FP32, patch slots (K, -x, +x, -y, +y),
// zeros outside the domain.  One 64-thread block per element; P = 2^k threads
// per row (P nn <= 64) share its dot product.
__global__ void k_patch_matvec(int64_t E, int nn, const int32_t* __restrict__ nbr, const float* __restrict__ A,
                               const double* __restrict__ r, double* __restrict__ y) {
  const int64_t K = blockIdx.x;
  if (K >= E) return;
  const int nc = 5 * nn;
  __shared__ double rp[320];
  for (int t = threadIdx.x; t < nc; t += blockDim.x) {
    const int slot = t / nn;
    const int64_t el = slot == 0 ? K : (int64_t)nbr[K * 4 + (slot - 1)];
    rp[t] = el >= 0 ? r[el * nn + (t % nn)] : 0.0;
  }
  __syncthreads();
  int P = 1;
  while (2 * P * nn <= 64) P *= 2;
  const int i = threadIdx.x / P, q = threadIdx.x % P;
  double acc = 0.0;
  if (i < nn) {
    const float* a = A + (K * nn + i) * (int64_t)nc;
    for (int j = q; j < nc; j += P) acc += (double)a[j] * rp[j];
  }
  for (int off = 1; off < P; off <<= 1) acc += __shfl_xor(acc, off, 64);
  if (i < nn && q == 0) y[K * nn + i] = r[K * nn + i] + acc;
}
// For each listed element K (2D quadrilaterals, one variable): the patch is K
// and its four face neighbours in local-face order (-x, +x, -y, +y); missing
// neighbours contribute zeros.  Features: [r patch / s (5 nn) | log kappa patch
// (5 nn) | b patch (5 x 2 nn)], s = ||r patch||_2 + 1e-300.  Target rows (when
// e is given): e on K / s.
__global__ void k_gather_patches(int64_t B, int64_t E, const int32_t* __restrict__ elems, int nn,
                                 const int32_t* __restrict__ nbr, const double* __restrict__ r,
                                 const double* __restrict__ aux, int naux, const double* __restrict__ e,
                                 float* __restrict__ X, float* __restrict__ Y, double* __restrict__ S) {
  const int64_t bidx = blockIdx.x;
  if (bidx >= B) return;
  const int64_t K = elems ? elems[bidx] : bidx;
  if (K < 0 || K >= E) {
    // an element index outside the mesh yields an all-zero sample (scale 0) instead of a stray read
    for (int t = threadIdx.x; t < 20 * nn; t += blockDim.x) X[bidx * 20 * nn + t] = 0.f;
    if (Y && e)
      for (int j = threadIdx.x; j < nn; j += blockDim.x) Y[bidx * nn + j] = 0.f;
    if (S && threadIdx.x == 0) S[bidx] = 0.0;
    return;
  }
  __shared__ double red[64];
  __shared__ int64_t pe[5];
  if (threadIdx.x < 5) {
    if (threadIdx.x == 0) pe[0] = K;
    else {
      const int32_t nb = nbr[K * 4 + (threadIdx.x - 1)];
      pe[threadIdx.x] = nb >= 0 ? nb : -1;
    }
  }
  __syncthreads();
  const int npatch = 5 * nn;
  double ss = 0.0;
  for (int t = threadIdx.x; t < npatch; t += blockDim.x) {
    const int64_t el = pe[t / nn];
    const double val = el >= 0 ? r[el * nn + (t % nn)] : 0.0;
    ss += val * val;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_down(ss, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += red[w];
    red[63] = sqrt(t) + 1e-300;
  }
  __syncthreads();
  const double sc = red[63];
  const int in_dim = npatch * 4;   // r, log kappa, b_x, b_y
  float* Xr = X + bidx * in_dim;
  for (int t = threadIdx.x; t < npatch; t += blockDim.x) {
    const int64_t el = pe[t / nn];
    Xr[t] = el >= 0 ? (float)(r[el * nn + (t % nn)] / sc) : 0.f;
    patch_coefs(Xr + npatch, t, el, nn, aux, naux);
  }
  if (Y && e)
    for (int j = threadIdx.x; j < nn; j += blockDim.x) Y[bidx * nn + j] = (float)(e[K * nn + j] / sc);
  if (S && threadIdx.x == 0) S[bidx] = sc;
}

// z_K += s_K * y_K  (network output rescaled onto the element)
__global__ void k_add_scaled_output(int64_t E, int nn, const float* __restrict__ Yo, const double* __restrict__ S,
                                    double* __restrict__ z, int composite) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E * nn) return;
  const double val = (double)Yo[t] * S[t / nn];
  z[t] = composite ? z[t] + val : val;
}

__global__ void k_count_nonfinite(int64_t n, const double* __restrict__ z, int* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(z[i])) atomicAdd(cnt, 1);
}

// Adam step (when lr > 0) and the loss to the host (synchronizes)
static ldg_status adam_and_loss(MlpNet& net, float lr, float* loss_host, hipStream_t s) {
  MlpNet* n = &net;
  if (lr > 0.0f) {
    n->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)n->t), c2 = 1.0f - powf(b2, (float)n->t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n->nparams + 255) / 256)), dim3(256), 0, s, n->nparams, lr, b1, b2,
                       1e-8f, c1, c2, n->params, n->grads, n->m1, n->m2);
    LDG_TRY(hipGetLastError());
  }
  if (loss_host) {
    LDG_TRY(hipMemcpyAsync(loss_host, n->loss_dev, sizeof(float), hipMemcpyDeviceToHost, s));
    LDG_TRY(hipStreamSynchronize(s));
  }
  return LDG_OK;
}

}  // namespace ldg

using namespace ldg;

struct ldg_mlp_s : public MlpNet {};

extern "C" {

ldg_status ldg_mlp_create(int in_dim, int width, int out_dim, int nlayers, int use_bf16, ldg_mlp* out) {
  LDG_ENTER();
  if (!out || in_dim <= 0 || width <= 0 || out_dim <= 0) { set_error("bad MLP sizes"); return LDG_EINVAL; }
  if (nlayers != 3) { set_error("the MLP has 3 layers"); return LDG_EUNSUPPORTED; }
  auto* n = new ldg_mlp_s();
  n->in_dim = in_dim; n->width = width; n->out_dim = out_dim; n->bf16 = use_bf16 != 0;
  int64_t o = 0;
  const int64_t sz[6] = {(int64_t)width * in_dim, width, (int64_t)width * width, width, (int64_t)out_dim * width, out_dim};
  for (int i = 0; i < 6; ++i) { n->off[i] = o; o += sz[i]; }
  n->nparams = o;
  hipError_t e = hipMalloc((void**)&n->params, sizeof(float) * o);
  if (e == hipSuccess) e = hipMalloc((void**)&n->grads, sizeof(float) * o);
  if (e == hipSuccess) e = hipMalloc((void**)&n->m1, sizeof(float) * o);
  if (e == hipSuccess) e = hipMalloc((void**)&n->m2, sizeof(float) * o);
  if (e == hipSuccess) e = hipMalloc((void**)&n->loss_dev, sizeof(float));
  if (e == hipSuccess) e = hipMemset(n->params, 0, sizeof(float) * o);
  if (e == hipSuccess) e = hipMemset(n->m1, 0, sizeof(float) * o);
  if (e == hipSuccess) e = hipMemset(n->m2, 0, sizeof(float) * o);
  if (e != hipSuccess) { set_error("MLP allocation failed"); delete n; return LDG_ENOMEM; }
  *out = n;
  return LDG_OK;
}

ldg_status ldg_mlp_destroy(ldg_mlp n) {
  if (!n) return LDG_OK;
  float* bufs[] = {n->params, n->grads, n->m1, n->m2, n->loss_dev, n->H1, n->H2, n->Yo, n->dY, n->dH2, n->dH1, n->part};
  for (float* b : bufs) if (b) (void)hipFree(b);
  delete n;
  return LDG_OK;
}

// HOST float params [nparams] packed W1 b1 W2 b2 W3 b3 (row-major W[out][in]); resets Adam
ldg_status ldg_mlp_set_params(ldg_mlp n, const float* host_params) {
  LDG_ENTER();
  if (!n || !host_params) { set_error("null argument"); return LDG_EINVAL; }
  LDG_TRY(hipMemcpy(n->params, host_params, sizeof(float) * n->nparams, hipMemcpyHostToDevice));
  LDG_TRY(hipMemset(n->m1, 0, sizeof(float) * n->nparams));
  LDG_TRY(hipMemset(n->m2, 0, sizeof(float) * n->nparams));
  n->t = 0;
  return LDG_OK;
}

ldg_status ldg_mlp_get_params(ldg_mlp n, float* host_params, float* host_grads) {
  LDG_ENTER();
  if (!n) { set_error("null argument"); return LDG_EINVAL; }
  if (host_params) LDG_TRY(hipMemcpy(host_params, n->params, sizeof(float) * n->nparams, hipMemcpyDeviceToHost));
  if (host_grads) LDG_TRY(hipMemcpy(host_grads, n->grads, sizeof(float) * n->nparams, hipMemcpyDeviceToHost));
  return LDG_OK;
}

ldg_status ldg_mlp_forward(ldg_mlp n, const float* X, int64_t B, float* Y, void* stream) {
  LDG_ENTER();
  if (!n || !X || !Y || B <= 0 || B >= (1ll << 31)) { set_error("bad arguments"); return LDG_EINVAL; }
  return mlp_forward(*n, X, B, Y, (hipStream_t)stream);
}

ldg_status ldg_mlp_forward_noalloc(ldg_mlp n, const float* X, int64_t B, float* Y, void* stream) {
  LDG_ENTER();
  if (!n || !X || !Y || B <= 0 || B >= (1ll << 31)) { set_error("bad arguments"); return LDG_EINVAL; }
  const int64_t need = 2 * B * (int64_t)n->width;
  if (need > kScratchFloats) {
    set_error("ldg_mlp_forward_noalloc: 2 * B * width = " + std::to_string(need) + " floats exceeds the fixed " +
              std::to_string(kScratchFloats) + "-float scratch (B <= " + std::to_string(kScratchFloats / (2 * n->width)) +
              " at this width); use ldg_mlp_forward");
    return LDG_EINVAL;
  }
  float* sc = nullptr;
  ldg_status st = scratch_address(&sc);
  if (st != LDG_OK) return st;
  // every entry of H1 and H2 that layer 2 and 3 read is written by layers 1 and 2 first
  return mlp_layers(*n, X, B, sc, sc + B * (int64_t)n->width, Y, (hipStream_t)stream, false);
}

// forward + MSE + backward (+ Adam when lr > 0); loss to HOST *loss_host (synchronizes)
ldg_status ldg_mlp_train_step(ldg_mlp n, const float* X, const float* Y, int64_t B, float lr, float* loss_host,
                              void* stream) {
  LDG_ENTER();
  if (!n || !X || !Y || B <= 0 || B >= (1ll << 31)) { set_error("bad arguments"); return LDG_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  // the work buffers (net.Yo among them) exist only after ensure_cap
  ldg_status st = ensure_cap(*n, B, s);
  if (st == LDG_OK) st = mlp_forward(*n, X, B, n->Yo, s);
  if (st == LDG_OK) st = mlp_backward(*n, X, Y, B, s);
  if (st != LDG_OK) return st;
  return adam_and_loss(*n, lr, loss_host, s);
}

// the linear form's training step: the network reads the coefficient features
// X[b][5 nn : 20 nn] and its output, viewed as A_b [nn][5 nn], multiplies the
// residual patch X[b][0 : 5 nn]; mean squared error of A_b r_b against Y[b]
ldg_status ldg_mlp_train_step_bilinear(ldg_mlp n, const float* X, const float* Y, int64_t B, float lr,
                                       float* loss_host, void* stream) {
  LDG_ENTER();
  if (!n || !X || !Y || B <= 0 || B >= (1ll << 31)) { set_error("bad arguments"); return LDG_EINVAL; }
  const int nn = n->in_dim / 15;
  if (n->in_dim % 15 != 0 || nn < 1 || nn > 64 || n->out_dim != 5 * nn * nn) {
    set_error("the linear form needs in_dim = 15 nn (coefficient patch) and out_dim = 5 nn^2 (an nn x 5 nn map)");
    return LDG_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int64_t ldx = 20 * (int64_t)nn;
  ldg_status st = ensure_cap(*n, B, s);
  if (st == LDG_OK) st = mlp_forward(*n, X + 5 * nn, B, n->Yo, s, ldx);
  if (st != LDG_OK) return st;
  hipLaunchKernelGGL(k_zero_f, dim3(1), dim3(64), 0, s, (int64_t)1, n->loss_dev);
  hipLaunchKernelGGL(k_bilinear_loss, dim3((unsigned)B), dim3(64), sizeof(float) * 6 * nn, s, B, nn, X, ldx, n->Yo, Y,
                     1.0f / (float)(B * nn), n->dY, n->loss_dev);
  LDG_TRY(hipGetLastError());
  if ((st = mlp_backward_dy(*n, X + 5 * nn, ldx, B, s)) != LDG_OK) return st;
  return adam_and_loss(*n, lr, loss_host, s);
}


ldg_status ldg_mlp_gather_patches(ldg_model md, const double* r, const double* e_target, const int32_t* elem_idx,
                                  int64_t B, float* X, float* Y, double* S, void* stream) {
  LDG_ENTER();
  if (!md || !r || !X || B <= 0) { set_error("bad arguments"); return LDG_EINVAL; }
  if (md->mesh->nd != 2 || md->ncu != 1) { set_error("element patches are defined for 2D scalar models"); return LDG_EUNSUPPORTED; }
  if (md->naux != 0 && md->naux != 3) { set_error("patch features need aux = [kappa, b_x, b_y]"); return LDG_EUNSUPPORTED; }
  hipLaunchKernelGGL(k_gather_patches, dim3((unsigned)B), dim3(64), 0, (hipStream_t)stream, B, md->mesh->E, elem_idx,
                     md->mesh->nn,
                     md->mesh->d_nbr, r, md->aux, md->naux, e_target, X, Y, S);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

}  // extern "C"

// ---------------------------------------------------------- preconditioner --
namespace ldg {

struct MlpPrecondData {
  Model* md;
  MlpNet* net;
  ldg_precond_s* bj;
  int composite;             // 0: s N(...), 1: B^-1 r + s N(...), 2: linear form B^-1 (r + A patch(r))
  float* X = nullptr;
  double* S = nullptr;
  float* Yo = nullptr;
  int* cnt = nullptr;
  float* Amap = nullptr;     // linear form: A [E][nn][5 nn]
  double* ybuf = nullptr;    // linear form: r + A patch(r)
};

ldg_status precond_apply_impl(ldg_precond_s* pc, const double* r, double* z, hipStream_t s);

ldg_status mlp_precond_apply(void* data, const double* r, double* z, hipStream_t s) {
  auto* d = (MlpPrecondData*)data;
  Model& md = *d->md;
  const int64_t E = md.mesh->E;
  const int nn = md.mesh->nn;
  ldg_status st;
  if (d->composite == 2) {
    hipLaunchKernelGGL(k_patch_matvec, dim3((unsigned)E), dim3(64), 0, s, E, nn, md.mesh->d_nbr, d->Amap, r, d->ybuf);
    LDG_TRY(hipGetLastError());
    return precond_apply_impl(d->bj, d->ybuf, z, s);
  }
  if (d->composite && d->bj) {
    st = precond_apply_impl(d->bj, r, z, s);
    if (st != LDG_OK) return st;
  }
  hipLaunchKernelGGL(k_gather_patches, dim3((unsigned)E), dim3(64), 0, s, E, E, (const int32_t*)nullptr, nn,
                     md.mesh->d_nbr, r, md.aux, md.naux, (const double*)nullptr, d->X, (float*)nullptr, d->S);
  LDG_TRY(hipGetLastError());
  st = mlp_forward(*d->net, d->X, E, d->Yo, s);
  if (st != LDG_OK) return st;
  hipLaunchKernelGGL(k_add_scaled_output, dim3((unsigned)((E * nn + 255) / 256)), dim3(256), 0, s, E, nn, d->Yo, d->S,
                     z, d->composite && d->bj ? 1 : 0);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

ldg_status mlp_precond_count_nonfinite(void* data, const double* z, int64_t n, int* host_cnt, hipStream_t s) {
  auto* d = (MlpPrecondData*)data;
  if (zero_int(d->cnt, s) != LDG_OK) return LDG_EDEVICE;
  hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, z, d->cnt);
  LDG_TRY(hipGetLastError());
  LDG_TRY(hipMemcpyAsync(host_cnt, d->cnt, sizeof(int), hipMemcpyDeviceToHost, s));
  LDG_TRY(hipStreamSynchronize(s));
  return LDG_OK;
}

void mlp_precond_destroy(void* data);

// The linear form: the coefficient features of every element, the network's
// output A_K for each (on the null stream, which this call synchronizes).
static ldg_status linear_form_setup(MlpPrecondData* d) {
  Model& md = *d->md;
  const int64_t E = md.mesh->E;
  const int nn = md.mesh->nn;
  float* C = nullptr;
  LDG_TRY(hipMalloc((void**)&d->Amap, sizeof(float) * E * 5 * nn * nn));
  LDG_TRY(hipMalloc((void**)&d->ybuf, sizeof(double) * E * nn));
  LDG_TRY(hipMalloc((void**)&C, sizeof(float) * E * 15 * nn));
  hipLaunchKernelGGL(k_coef_patches, dim3((unsigned)E), dim3(64), 0, nullptr, E, nn, md.mesh->d_nbr, md.aux, md.naux, C);
  ldg_status st = LDG_OK;
  if (hipGetLastError() != hipSuccess) { set_error("coefficient patch launch failed"); st = LDG_EDEVICE; }
  if (st == LDG_OK) st = mlp_forward(*d->net, C, E, d->Amap, nullptr);
  const hipError_t e = hipStreamSynchronize(nullptr);
  (void)hipFree(C);
  if (st == LDG_OK && e != hipSuccess) { set_error(std::string("linear form set-up: ") + hipGetErrorString(e)); st = LDG_EDEVICE; }
  return st;
}

void* mlp_precond_create(Model* md, MlpNet* net, ldg_precond_s* bj, int composite, ldg_status* status) {
  auto* d = new MlpPrecondData();
  d->md = md; d->net = net; d->bj = bj; d->composite = composite;
  const int64_t E = md->mesh->E;
  const int nn = md->mesh->nn;
  *status = LDG_OK;
  if (composite == 2) {
    *status = linear_form_setup(d);
    if (*status == LDG_OK && hipMalloc((void**)&d->cnt, sizeof(int)) != hipSuccess) {
      set_error("allocation failed");
      *status = LDG_ENOMEM;
    }
    if (*status != LDG_OK) {
      mlp_precond_destroy(d);
      return nullptr;
    }
    return d;
  }
  *status = LDG_ENOMEM;
  if (hipMalloc((void**)&d->X, sizeof(float) * E * net->in_dim) != hipSuccess ||
      hipMalloc((void**)&d->S, sizeof(double) * E) != hipSuccess ||
      hipMalloc((void**)&d->Yo, sizeof(float) * E * nn) != hipSuccess ||
      hipMalloc((void**)&d->cnt, sizeof(int)) != hipSuccess) {
    set_error("allocation failed");
    mlp_precond_destroy(d);
    return nullptr;
  }
  *status = LDG_OK;
  return d;
}

void mlp_precond_destroy(void* data) {
  auto* d = (MlpPrecondData*)data;
  if (!d) return;
  (void)hipFree(d->X); (void)hipFree(d->S); (void)hipFree(d->Yo); (void)hipFree(d->cnt);
  (void)hipFree(d->Amap); (void)hipFree(d->ybuf);
  delete d;
}

ldg_precond_s* mlp_precond_fallback(void* data) { return ((MlpPrecondData*)data)->bj; }

void mlp_dims(const MlpNet* net, int* in_dim, int* out_dim) {
  *in_dim = net->in_dim;
  *out_dim = net->out_dim;
}

}  // namespace ldg
