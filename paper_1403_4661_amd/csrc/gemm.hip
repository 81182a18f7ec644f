// Batched FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
// One workgroup (4 waves) computes a 64 x 64 tile of C for one descriptor;
// wave w owns rows [16w, 16w+16) and all 64 columns as four 16 x 16 MFMA
// accumulators.  Operand layout of the 16x16x4 f64 MFMA: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register v of lane l
// holds D[l / 16 + 4 v][l % 16].  A and B tiles (64 x 16 and 16 x 64) are
// staged through LDS; loads follow whichever stride is unit so that global
// reads are coalesced for both storage orders.  Out-of-range rows, columns and k are zero-filled,
// so any M, N, K >= 0 is valid.

#include "common.hpp"

namespace osht {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int TM = 64, TN = 64, TK = 16, PAD = 2;
constexpr int EA = TM * TK / 256, EB = TK * TN / 256;  // elements per thread per tile (4)

// Element t (0..3) of this thread in a 64 x 16 A tile / 16 x 64 B tile.
// ARF: A rows contiguous (column-major A); BCF: B columns contiguous.
template <bool ARF>
__device__ __forceinline__ void a_coord(int t, int& i, int& kk) {
  if (ARF) { i = threadIdx.x & 63; kk = (threadIdx.x >> 6) + 4 * t; }
  else { kk = threadIdx.x & 15; i = (threadIdx.x >> 4) + 16 * t; }
}
template <bool BCF>
__device__ __forceinline__ void b_coord(int t, int& kk, int& j) {
  if (BCF) { j = threadIdx.x & 63; kk = (threadIdx.x >> 6) + 4 * t; }
  else { kk = threadIdx.x & 15; j = (threadIdx.x >> 4) + 16 * t; }
}

template <bool ARF, bool BCF>
__device__ __forceinline__ void load_tile(const GemmDesc& d, int m0, int n0, int k0, double* ra, double* rb) {
#pragma unroll
  for (int t = 0; t < EA; ++t) {
    int i, kk;
    a_coord<ARF>(t, i, kk);
    const int gi = m0 + i, gk = k0 + kk;
    ra[t] = (gi < d.M && gk < d.K) ? d.A[(int64_t)gi * d.sAr + (int64_t)gk * d.sAc] : 0.0;
  }
#pragma unroll
  for (int t = 0; t < EB; ++t) {
    int kk, j;
    b_coord<BCF>(t, kk, j);
    const int gk = k0 + kk, gj = n0 + j;
    rb[t] = (gk < d.K && gj < d.N) ? d.B[(int64_t)gk * d.sBr + (int64_t)gj * d.sBc] : 0.0;
  }
}

template <bool ARF, bool BCF>
__device__ __forceinline__ void store_tile(double (*As)[TM + PAD], double (*Bs)[TN + PAD], const double* ra,
                                           const double* rb) {
#pragma unroll
  for (int t = 0; t < EA; ++t) {
    int i, kk;
    a_coord<ARF>(t, i, kk);
    As[kk][i] = ra[t];
  }
#pragma unroll
  for (int t = 0; t < EB; ++t) {
    int kk, j;
    b_coord<BCF>(t, kk, j);
    Bs[kk][j] = rb[t];
  }
}

// Software-pipelined: the global loads of k-tile t+1 are issued into
// registers before the MFMAs of tile t run from LDS; LDS is double
// buffered, so one barrier per k-tile suffices.
template <bool ARF, bool BCF>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const GemmDesc* __restrict__ descs,
                                                       const GemmTask* __restrict__ tasks) {
  const GemmTask t = tasks[blockIdx.x];
  const GemmDesc d = descs[t.desc];
  const int m0 = t.mt * TM, n0 = t.nt * TN;
  __shared__ double As[2][TK][TM + PAD];
  __shared__ double Bs[2][TK][TN + PAD];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  dbl4 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = dbl4{0.0, 0.0, 0.0, 0.0};
  double ra[EA], rb[EB];
  const int nt = (d.K + TK - 1) / TK;
  if (nt > 0) {
    load_tile<ARF, BCF>(d, m0, n0, 0, ra, rb);
    store_tile<ARF, BCF>(As[0], Bs[0], ra, rb);
  }
  __syncthreads();
  for (int kt = 0; kt < nt; ++kt) {
    const int p = kt & 1;
    const bool more = kt + 1 < nt;
    if (more) load_tile<ARF, BCF>(d, m0, n0, (kt + 1) * TK, ra, rb);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const double a = As[p][kk + (lane >> 4)][wave * 16 + (lane & 15)];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const double b = Bs[p][kk + (lane >> 4)][nb * 16 + (lane & 15)];
        acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[nb], 0, 0, 0);
      }
    }
    if (more) store_tile<ARF, BCF>(As[p ^ 1], Bs[p ^ 1], ra, rb);
    __syncthreads();
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + wave * 16 + (lane >> 4) + 4 * v;  // f64 16x16x4 D layout
      const int col = n0 + nb * 16 + (lane & 15);
      if (row < d.M && col < d.N) {
        double* cp = d.C + (int64_t)row * d.sCr + (int64_t)col * d.sCc;
        double r = d.alpha * acc[nb][v];
        if (d.beta != 0.0) r += d.beta * (*cp);
        *cp = r;
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

void launch_gemm_f64(const GemmDesc* d_desc, const GemmTask* d_task, int ntask, bool a_rowfast, bool b_colfast,
                     hipStream_t st) {
  if (ntask <= 0) return;
  if (a_rowfast && b_colfast)
    hipLaunchKernelGGL((gemm_f64_kernel<true, true>), dim3(ntask), dim3(256), 0, st, d_desc, d_task);
  else if (a_rowfast)
    hipLaunchKernelGGL((gemm_f64_kernel<true, false>), dim3(ntask), dim3(256), 0, st, d_desc, d_task);
  else if (b_colfast)
    hipLaunchKernelGGL((gemm_f64_kernel<false, true>), dim3(ntask), dim3(256), 0, st, d_desc, d_task);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<false, false>), dim3(ntask), dim3(256), 0, st, d_desc, d_task);
  OSHT_HIP(hipGetLastError());
}

}  // namespace osht
