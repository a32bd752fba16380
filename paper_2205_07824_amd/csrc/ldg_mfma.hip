// Mixed-precision Jacobian-vector product of the linear models with the
// element-volume contractions on MFMA: bf16 or fp16 operands, fp32
// accumulation.  The reference-gradient operator of one element,
// G = [D_1; ...; D_d] ((d nn) x nn, D_j = I x .. x D x .. x I), is applied to
// all elements at once as one GEMM (elements are the batch dimension):
//     dU[e][(j,i)] = sum_m v[e][m] G[(j,i)][m]
// and the weak divergence as its transpose:
//     out[e][i]  -= sum_{(j,m)} F[e][(j,m)] G[(j,m)][i].
// Face traces, lifting, the metric transform and the flux stay in the FP32
// operator kernels (k_grad / k_resid with external contractions).
#include <vector>

#include "ldg_internal.hpp"

namespace ldg {

ldg_status op_grad_ext(const Model& md, const double* u, const float* du, float* q, hipStream_t s);
ldg_status op_resid_ext(const Model& md, const TimeDev& t, const double* u, const float* q, float* Fout,
                        double* out, hipStream_t s);

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 h16x4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline short to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// C(m,n) (=|-=) sum_k A(m,k) B(k,n), A row-major [M][K] (double or float), B row-major [K][N] float.
// 64 x 64 tile per 256 threads, 2x2 MFMA 16x16x16 tiles per wave.
template <class TA, class TC, bool SUB, bool F16>
__global__ void __launch_bounds__(256) k_mfma_gemm(int M, int N, int K, const TA* __restrict__ A,
                                                   const float* __restrict__ B, TC* __restrict__ C) {
  __shared__ float As[64][17];
  __shared__ float Bs[16][65];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, kg = lane >> 4;
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * 256;
      const int am = e >> 4, ak = e & 15;
      As[am][ak] = (m0 + am < M && k0 + ak < K) ? (float)A[(int64_t)(m0 + am) * K + k0 + ak] : 0.0f;
      const int bk = e >> 6, bn = e & 63;
      Bs[bk][bn] = (k0 + bk < K && n0 + bn < N) ? B[(int64_t)(k0 + bk) * N + n0 + bn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        if constexpr (F16) {
          h16x4 af, bf;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            af[i] = (_Float16)As[wr + a * 16 + li][kg * 4 + i];
            bf[i] = (_Float16)Bs[kg * 4 + i][wc + b * 16 + li];
          }
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16f16(af, bf, acc[a][b], 0, 0, 0);
        } else {
          s16x4 af, bf;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            af[i] = to_bf16(As[wr + a * 16 + li][kg * 4 + i]);
            bf[i] = to_bf16(Bs[kg * 4 + i][wc + b * 16 + li]);
          }
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bf, acc[a][b], 0, 0, 0);
        }
      }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gm = m0 + wr + a * 16 + kg * 4 + i, gn = n0 + wc + b * 16 + li;
        if (gm < M && gn < N) {
          if constexpr (SUB) C[(int64_t)gm * N + gn] -= (TC)acc[a][b][i];
          else C[(int64_t)gm * N + gn] = (TC)acc[a][b][i];
        }
      }
}

template <class TA, class TC, bool SUB>
static ldg_status gemm_launch(bool f16, int M, int N, int K, const TA* A, const float* B, TC* C, hipStream_t s) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  if (f16) hipLaunchKernelGGL((k_mfma_gemm<TA, TC, SUB, true>), grid, dim3(256), 0, s, M, N, K, A, B, C);
  else hipLaunchKernelGGL((k_mfma_gemm<TA, TC, SUB, false>), grid, dim3(256), 0, s, M, N, K, A, B, C);
  LDG_TRY(hipGetLastError());
  return LDG_OK;
}

// Operators of the two GEMMs, built once at model creation (linear models).
// The FP32 intermediates of a product use the model's workspace: dU and F
// share the FP64 linearization cache d_q (linear models never fill it; 2 NQ
// floats = NQ doubles), q goes to the tangent buffer d_dq.
struct MfmaWork {
  float* G = nullptr;    // [(d nn)][nn] reference-gradient operator
  float* GT = nullptr;   // [nn][(d nn)] its transpose (for the first GEMM's B operand)
};

ldg_status mfma_prepare(Model& md) {
  const Mesh& m = *md.mesh;
  const int nn = m.nn, d = m.nd, P1 = m.p1;
  std::vector<float> G((size_t)d * nn * nn, 0.0f), GT((size_t)nn * d * nn, 0.0f);
  for (int j = 0; j < d; ++j)
    for (int i = 0; i < nn; ++i)
      for (int mm = 0; mm < nn; ++mm) {
        int ai[3], am[3], ti = i, tm = mm;
        for (int k = 0; k < d; ++k) { ai[k] = ti % P1; ti /= P1; am[k] = tm % P1; tm /= P1; }
        bool same = true;
        for (int k = 0; k < d; ++k)
          if (k != j && ai[k] != am[k]) same = false;
        const float val = same ? (float)m.tab.D[ai[j]][am[j]] : 0.0f;
        G[((size_t)j * nn + i) * nn + mm] = val;
        GT[(size_t)mm * d * nn + (size_t)j * nn + i] = val;
      }
  auto* w = new MfmaWork();
  md.mfma = w;   // released by mfma_release, also on the error paths below
  LDG_TRY(hipMalloc((void**)&w->G, G.size() * 4));
  LDG_TRY(hipMalloc((void**)&w->GT, GT.size() * 4));
  LDG_TRY(hipMemcpy(w->G, G.data(), G.size() * 4, hipMemcpyHostToDevice));
  LDG_TRY(hipMemcpy(w->GT, GT.data(), GT.size() * 4, hipMemcpyHostToDevice));
  return LDG_OK;
}

void mfma_release(Model& md) {
  if (!md.mfma) return;
  (void)hipFree(md.mfma->G);
  (void)hipFree(md.mfma->GT);
  delete md.mfma;
  md.mfma = nullptr;
}

ldg_status op_mfma_jvp(const Model& md, const TimeDev& t, const double* v, double* out, bool fp16, hipStream_t s) {
  const MfmaWork* w = md.mfma;
  if (!w) { set_error("MFMA JVP operators missing (linear models build them at creation)"); return LDG_EUNSUPPORTED; }
  const Mesh& m = *md.mesh;
  const int nn = m.nn, d = m.nd;
  const int E = (int)m.E;
  float* dU = (float*)md.d_q;
  float* F = dU + (size_t)E * d * nn;
  float* q = (float*)md.d_dq;
  // reference gradient of v on MFMA: dU = V G^T  ([E][nn] x [nn][d nn])
  ldg_status st = gemm_launch<double, float, false>(fp16, E, d * nn, nn, v, w->GT, dU, s);
  if (st != LDG_OK) return st;
  // q = metric transform + lifting (FP32)
  st = op_grad_ext(md, v, dU, q, s);
  if (st != LDG_OK) return st;
  // fluxes, face terms, pointwise terms (FP32); contravariant flux to F
  st = op_resid_ext(md, t, v, q, F, out, s);
  if (st != LDG_OK) return st;
  // weak divergence on MFMA: out -= F G  ([E][d nn] x [d nn][nn])
  return gemm_launch<float, double, true>(fp16, E, nn, d * nn, F, w->G, out, s);
}

}  // namespace ldg
