// Block-Jacobi preconditioner: exact element diagonal blocks of the Jacobian by
// probing (one JVP per element colour and local unknown; elements of one colour
// are at face-graph distance >= 3, beyond the reach of the LDG stencil), batched
// Gauss-Jordan inversion with partial pivoting, and a batched block-matrix
// vector product as the apply (FP64 or FP32 storage).
#include <cmath>

#include "ldg_internal.hpp"

struct ldg_precond_s {
  int kind = 0;           // 0 block-Jacobi, 1 learned (MLP) composite
  void* mlp_data = nullptr;
  ldg::Model* md;
  int per_variable;
  ldg_precision prec;     // storage precision of the inverse blocks
  int nb;                 // block size
  int64_t nblocks;        // E (full) or E * ncu (per variable)
  void* inv = nullptr;    // [nblocks][nb][nb], transposed: inv[b][j][i] = (B_b^-1)[i][j]
  double* scratch = nullptr;  // assembled blocks [nblocks][nb][nb] row-major
  int* info = nullptr;        // singular-block counter (device)
  double a0 = 0.0;
};

namespace ldg {

__global__ void k_probe_set(int n, const int32_t* __restrict__ list, int NB, int j, double val,
                            double* __restrict__ v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) v[(int64_t)list[t] * NB + j] = val;
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

// In-place Gauss-Jordan inversion with row pivoting of one nb x nb block per
// work-group (A in LDS when it fits, otherwise in global memory), written out
// transposed in the storage precision.
template <class S>
__global__ void __launch_bounds__(256) k_gj_invert(int nb, double* __restrict__ blocks, S* __restrict__ inv,
                                                   int use_lds, int* __restrict__ info) {
  extern __shared__ double lds[];
  __shared__ int piv[128];
  __shared__ double fcol[128];
  __shared__ int pidx;
  __shared__ double bestv;
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
      if (tid == 0) { pidx = bi; bestv = bv; piv[k] = bi; }
    }
    __syncthreads();
    const int p = pidx;
    if (tid == 0 && !(bestv > 0.0)) atomicAdd(info, 1);
    if (p != k)
      for (int j = tid; j < nb; j += nt) {
        const double t = A[k * nb + j];
        A[k * nb + j] = A[p * nb + j];
        A[p * nb + j] = t;
      }
    __syncthreads();
    const double pv = A[k * nb + k];
    const double ipv = pv != 0.0 ? 1.0 / pv : 0.0;
    for (int i = tid; i < nb; i += nt) fcol[i] = (i == k) ? 0.0 : A[i * nb + k];
    __syncthreads();
    for (int j = tid; j < nb; j += nt) A[k * nb + j] = (j == k ? 1.0 : A[k * nb + j]) * ipv;
    __syncthreads();
    // rank-1 update of the other rows: thread (r0, j) owns column j of rows r0, r0 + rpp, ...
    if (r0 < rpp) {
      const double akj = A[k * nb + jc];
      for (int i = r0; i < nb; i += rpp) {
        if (i == k) continue;
        const double base = (jc == k) ? 0.0 : A[i * nb + jc];
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
  S* out = inv + b * (int64_t)nb * nb;
  if (r0 < rpp)
    for (int j = r0; j < nb; j += rpp) out[j * nb + jc] = (S)A[jc * nb + j];   // out[j][i] = A[i][j]
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
template <class S, int NB>
__global__ void __launch_bounds__(1024) k_bj_apply(int nb_rt, int64_t nblocks, int bpb, const S* __restrict__ inv,
                                                  const double* __restrict__ r, double* __restrict__ z) {
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
  z[b * nb + i] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// probe = LDG_FP32 for blocks that are stored in FP32 anyway (the probing JVPs
// then run in FP32 too)
static ldg_status assemble_blocks(Model& md, const ldg_time* t, const double* u_lin, int per_variable,
                                  double* blocks, ldg_precision probe, hipStream_t s) {
  Mesh& m = *md.mesh;
  const int NB = md.ncu * m.nn;
  const int64_t n = (int64_t)md.N();
  ldg_status st;
  if (!md.linear && md.kind != LDG_MODEL_EULER) {
    st = op_grad(md, u_lin, md.d_q, false, true, s);
    if (st != LDG_OK) return st;
    if (probe == LDG_FP32) {
      st = op_grad(md, u_lin, md.d_q32, true, true, s);
      if (st != LDG_OK) return st;
    }
  }
  double* v = md.d_tmp;
  double* Jv = md.d_tmp2;
  st = vec_fill(n, 0.0, v, s);
  if (st != LDG_OK) return st;
  for (int c = 0; c < m.ncolors; ++c) {
    const int cnt = (int)(m.color_off[c + 1] - m.color_off[c]);
    const int32_t* list = m.d_color_list + m.color_off[c];
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
    if (pc->prec == LDG_FP32)
      (void)hipFuncSetAttribute((const void*)k_gj_invert<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    else
      (void)hipFuncSetAttribute((const void*)k_gj_invert<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    (void)hipGetLastError();
  }
  if (nb > 128) { set_error("block size above 128"); return LDG_EUNSUPPORTED; }
  if (zero_int(pc->info, s) != LDG_OK) return LDG_EDEVICE;
  const int threads = 256;
  if (pc->prec == LDG_FP32)
    hipLaunchKernelGGL(k_gj_invert<float>, dim3((unsigned)pc->nblocks), dim3(threads), use_lds ? bytes : 0, s, nb,
                       pc->scratch, (float*)pc->inv, use_lds, pc->info);
  else
    hipLaunchKernelGGL(k_gj_invert<double>, dim3((unsigned)pc->nblocks), dim3(threads), use_lds ? bytes : 0, s, nb,
                       pc->scratch, (double*)pc->inv, use_lds, pc->info);
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
  ldg_status st = assemble_blocks(*pc->md, t, u_lin, pc->per_variable, pc->scratch,
                                  pc->prec == LDG_FP32 ? LDG_FP32 : LDG_FP64, s);
  if (st != LDG_OK) return st;
  return invert_blocks(pc, s);
}

ldg_status mlp_precond_apply(void* data, const double* r, double* z, hipStream_t s);
void* mlp_precond_create(Model* md, struct MlpNet* net, ldg_precond_s* bj, int composite);
void mlp_precond_destroy(void* data);

ldg_status precond_apply_impl(ldg_precond_s* pc, const double* r, double* z, hipStream_t s) {
  if (pc->kind == 1) return mlp_precond_apply(pc->mlp_data, r, z, s);
  const int nb = pc->nb;
  int bpb = 256 / nb;
  if (bpb < 1) bpb = 1;
  const unsigned grid = (unsigned)((pc->nblocks + bpb - 1) / bpb);
  const size_t sh = (size_t)bpb * nb * sizeof(double);
  const dim3 thr(bpb * nb);
  if (nb > 1024) { set_error("block-Jacobi blocks larger than 1024 rows"); return LDG_EUNSUPPORTED; }
  if (pc->prec == LDG_FP32) {
    if (nb == 64)
      hipLaunchKernelGGL((k_bj_apply<float, 64>), dim3(grid), thr, sh, s, nb, pc->nblocks, bpb, (const float*)pc->inv, r, z);
    else
      hipLaunchKernelGGL((k_bj_apply<float, 0>), dim3(grid), thr, sh, s, nb, pc->nblocks, bpb, (const float*)pc->inv, r, z);
  } else {
    if (nb == 64)
      hipLaunchKernelGGL((k_bj_apply<double, 64>), dim3(grid), thr, sh, s, nb, pc->nblocks, bpb, (const double*)pc->inv, r, z);
    else
      hipLaunchKernelGGL((k_bj_apply<double, 0>), dim3(grid), thr, sh, s, nb, pc->nblocks, bpb, (const double*)pc->inv, r, z);
  }
  LDG_TRY(hipGetLastError());
  return LDG_OK;
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
  if (factor_prec != LDG_FP64 && factor_prec != LDG_FP32) { set_error("factor precision must be FP64 or FP32"); return LDG_EINVAL; }
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
  hipError_t e = hipMalloc((void**)&pc->scratch, nel * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&pc->inv, nel * (factor_prec == LDG_FP32 ? sizeof(float) : sizeof(double)));
  if (e == hipSuccess) e = hipMalloc((void**)&pc->info, sizeof(int));
  if (e != hipSuccess) {
    hipFree(pc->scratch); hipFree(pc->inv); hipFree(pc->info);
    delete pc;
    set_error(std::string("block-Jacobi allocation: ") + hipGetErrorString(e));
    return LDG_ENOMEM;
  }
  ldg_status st = precond_rebuild(pc, t, u_lin, (hipStream_t)stream);
  if (st != LDG_OK) {
    hipFree(pc->scratch); hipFree(pc->inv); hipFree(pc->info);
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
  if (composite && !fallback_bj) { set_error("composite form needs the block-Jacobi part"); return LDG_EINVAL; }
  auto* pc = new ldg_precond_s();
  pc->kind = 1;
  pc->md = md;
  pc->nb = 0;
  pc->nblocks = 0;
  pc->mlp_data = mlp_precond_create(md, (MlpNet*)net, fallback_bj, composite);
  if (!pc->mlp_data) { delete pc; set_error("allocation failed"); return LDG_ENOMEM; }
  *out = pc;
  return LDG_OK;
}

ldg_status ldg_precond_destroy(ldg_precond pc) {
  LDG_ENTER();
  if (!pc) return LDG_OK;
  if (pc->kind == 1) { mlp_precond_destroy(pc->mlp_data); delete pc; return LDG_OK; }
  hipFree(pc->scratch); hipFree(pc->inv); hipFree(pc->info);
  delete pc;
  return LDG_OK;
}

}  // extern "C"
