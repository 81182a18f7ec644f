// Batched FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
// One workgroup (4 waves) computes a 64 x 64 tile of C for one descriptor;
// wave w owns rows [16w, 16w+16) and all 64 columns as four 16 x 16 MFMA
// accumulators.  Operand layout of the 16x16x4 f64 MFMA: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register v of lane l
// holds D[l / 16 + 4 v][l % 16].  A and B tiles (64 x 16 and 16 x 64) are staged through LDS;
// loads follow whichever stride is unit so that global reads are coalesced
// for both storage orders.  Out-of-range rows, columns and k are zero-filled,
// so any M, N, K >= 0 is valid.

#include "common.hpp"

namespace osht {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int TM = 64, TN = 64, TK = 16, PAD = 2;

__global__ __launch_bounds__(256) void gemm_f64_kernel(const GemmDesc* __restrict__ descs,
                                                       const GemmTask* __restrict__ tasks) {
  const GemmTask t = tasks[blockIdx.x];
  const GemmDesc d = descs[t.desc];
  const int m0 = t.mt * TM, n0 = t.nt * TN;
  __shared__ double As[TK][TM + PAD];
  __shared__ double Bs[TK][TN + PAD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  dbl4 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = dbl4{0.0, 0.0, 0.0, 0.0};
  const bool a_rowfast = (d.sAr == 1);
  const bool b_colfast = (d.sBc == 1);
  for (int k0 = 0; k0 < d.K; k0 += TK) {
#pragma unroll
    for (int e = tid; e < TM * TK; e += 256) {
      int i, kk;
      if (a_rowfast) { i = e % TM; kk = e / TM; } else { kk = e % TK; i = e / TK; }
      const int gi = m0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < d.M && gk < d.K) v = d.A[(int64_t)gi * d.sAr + (int64_t)gk * d.sAc];
      As[kk][i] = v;
    }
#pragma unroll
    for (int e = tid; e < TK * TN; e += 256) {
      int kk, j;
      if (b_colfast) { j = e % TN; kk = e / TN; } else { kk = e % TK; j = e / TK; }
      const int gk = k0 + kk, gj = n0 + j;
      double v = 0.0;
      if (gk < d.K && gj < d.N) v = d.B[(int64_t)gk * d.sBr + (int64_t)gj * d.sBc];
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const double a = As[kk + (lane >> 4)][wave * 16 + (lane & 15)];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const double b = Bs[kk + (lane >> 4)][nb * 16 + (lane & 15)];
        acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[nb], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + wave * 16 + (lane >> 4) + 4 * v;  // f64 16x16x4 D layout
      const int col = n0 + nb * 16 + (lane & 15);
      if (row < d.M && col < d.N) {
        double* c = d.C + (int64_t)row * d.sCr + (int64_t)col * d.sCc;
        double r = d.alpha * acc[nb][v];
        if (d.beta != 0.0) r += d.beta * (*c);
        *c = r;
      }
    }
  }
}

}  // namespace

void gemm_tasks(const std::vector<GemmDesc>& descs, std::vector<GemmTask>& tasks) {
  tasks.clear();
  for (size_t i = 0; i < descs.size(); ++i) {
    const int mt = (int)ceil_div(descs[i].M, TM), nt = (int)ceil_div(descs[i].N, TN);
    for (int a = 0; a < mt; ++a)
      for (int b = 0; b < nt; ++b) tasks.push_back(GemmTask{(int32_t)i, a, b, 0});
  }
}

void launch_gemm_f64(const GemmDesc* d_desc, const GemmTask* d_task, int ntask, hipStream_t st) {
  if (ntask <= 0) return;
  hipLaunchKernelGGL(gemm_f64_kernel, dim3(ntask), dim3(256), 0, st, d_desc, d_task);
  OSHT_HIP(hipGetLastError());
}

}  // namespace osht
