// Batched GEMM on CDNA4 matrix cores for the order-wise applies.
//
// C(M x N) = alpha * A(M x K) * B(K x N) + beta * C, with C and B in FP64
// and A (the plan's matrix: A_m, Q_m or their transposes) in FP64 or FP32.
//
// One workgroup (4 waves) computes a 64 x 64 tile of C for one descriptor;
// wave w owns rows [16w, 16w+16) and all 64 columns as four 16 x 16 MFMA
// accumulators.  A and B tiles (64 x 16 and 16 x 64) are staged through LDS;
// global loads follow whichever stride is unit, so reads are coalesced for
// both storage orders.  Out-of-range rows, columns and k are zero-filled, so
// any M, N, K >= 0 is valid.
//
// FP64 path: v_mfma_f64_16x16x4f64.  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register v of lane l holds
// D[l / 16 + 4 v][l % 16].
// FP32 path: v_mfma_f32_16x16x4f32 on A (stored FP32) and B rounded to FP32
// when staged.  Same operand layout; accumulator register v of lane l holds
// D[4 (l / 16) + v][l % 16].  Each 16-deep k-tile is accumulated in FP32 by
// the matrix core and then added into an FP64 running sum, so the FP32
// accumulation error is that of a 16-term sum whatever K is.
//
// The Role parameter only names the kernel symbol (inverse apply, forward
// apply, correction, adjoints, plan construction) so that per-kernel
// profiles separate the launches.

#include "common.hpp"

namespace osht {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

struct RolePlan {};
struct RoleApplyInverse {};
struct RoleApplyForward {};
struct RoleCorrection {};
struct RoleAdjoint {};

namespace {

constexpr int TM = 64, TN = 64, TK = 16;
constexpr int EA = TM * TK / 256, EB = TK * TN / 256;  // elements per thread per tile (4)

// LDS row padding: FP64 rows of 66 doubles; FP32 rows of 80 floats, so the
// four 16-lane groups of an operand read hit disjoint bank halves.
template <class T> struct Pad;
template <> struct Pad<double> { static constexpr int v = 2; };
template <> struct Pad<float> { static constexpr int v = 16; };

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

template <bool ARF, bool BCF, class T>
__device__ __forceinline__ void load_tile(const GemmDesc& d, const T* __restrict__ A, int m0, int n0, int k0, T* ra,
                                          T* rb) {
#pragma unroll
  for (int t = 0; t < EA; ++t) {
    int i, kk;
    a_coord<ARF>(t, i, kk);
    const int gi = m0 + i, gk = k0 + kk;
    ra[t] = (gi < d.M && gk < d.K) ? A[(int64_t)gi * d.sAr + (int64_t)gk * d.sAc] : T(0);
  }
#pragma unroll
  for (int t = 0; t < EB; ++t) {
    int kk, j;
    b_coord<BCF>(t, kk, j);
    const int gk = k0 + kk, gj = n0 + j;
    rb[t] = (gk < d.K && gj < d.N) ? T(d.B[(int64_t)gk * d.sBr + (int64_t)gj * d.sBc]) : T(0);
  }
}

template <bool ARF, bool BCF, class T, int P>
__device__ __forceinline__ void store_tile(T (*As)[TM + P], T (*Bs)[TN + P], const T* ra, const T* rb) {
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
template <bool ARF, bool BCF, class T, class Role>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmDesc* __restrict__ descs,
                                                   const GemmTask* __restrict__ tasks) {
  constexpr int P = Pad<T>::v;
  constexpr bool F64 = sizeof(T) == 8;
  const GemmTask t = tasks[blockIdx.x];
  const GemmDesc d = descs[t.desc];
  const T* __restrict__ A = static_cast<const T*>(d.A);
  const int m0 = t.mt * TM, n0 = t.nt * TN;
  __shared__ T As[2][TK][TM + P];
  __shared__ T Bs[2][TK][TN + P];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  dbl4 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = dbl4{0.0, 0.0, 0.0, 0.0};
  T ra[EA], rb[EB];
  const int nt = (d.K + TK - 1) / TK;
  if (nt > 0) {
    load_tile<ARF, BCF, T>(d, A, m0, n0, 0, ra, rb);
    store_tile<ARF, BCF, T, P>(As[0], Bs[0], ra, rb);
  }
  __syncthreads();
  for (int kt = 0; kt < nt; ++kt) {
    const int p = kt & 1;
    const bool more = kt + 1 < nt;
    if (more) load_tile<ARF, BCF, T>(d, A, m0, n0, (kt + 1) * TK, ra, rb);
    if constexpr (F64) {
#pragma unroll
      for (int kk = 0; kk < TK; kk += 4) {
        const double a = As[p][kk + (lane >> 4)][wave * 16 + (lane & 15)];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const double b = Bs[p][kk + (lane >> 4)][nb * 16 + (lane & 15)];
          acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[nb], 0, 0, 0);
        }
      }
    } else {
      flt4 c[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) c[nb] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < TK; kk += 4) {
        const float a = As[p][kk + (lane >> 4)][wave * 16 + (lane & 15)];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const float b = Bs[p][kk + (lane >> 4)][nb * 16 + (lane & 15)];
          c[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[nb], 0, 0, 0);
        }
      }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[nb][v] += (double)c[nb][v];
    }
    if (more) store_tile<ARF, BCF, T, P>(As[p ^ 1], Bs[p ^ 1], ra, rb);
    __syncthreads();
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + wave * 16 + (F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
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

template <bool ARF, bool BCF, class T, class Role>
void launch(const GemmDesc* d_desc, const GemmTask* d_task, int ntask, hipStream_t st) {
  hipLaunchKernelGGL((gemm_kernel<ARF, BCF, T, Role>), dim3(ntask), dim3(256), 0, st, d_desc, d_task);
}

template <class T>
void launch_role(GemmRole role, const GemmDesc* d_desc, const GemmTask* d_task, int ntask, hipStream_t st) {
  switch (role) {
    case GemmRole::ApplyInverse: launch<true, true, T, RoleApplyInverse>(d_desc, d_task, ntask, st); break;
    case GemmRole::ApplyForward: launch<true, true, T, RoleApplyForward>(d_desc, d_task, ntask, st); break;
    case GemmRole::Correction: launch<true, true, T, RoleCorrection>(d_desc, d_task, ntask, st); break;
    case GemmRole::Adjoint: launch<false, true, T, RoleAdjoint>(d_desc, d_task, ntask, st); break;
    default: throw Error{OSHT_EINVAL, "bad GEMM role"};
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

void launch_gemm(GemmRole role, bool fp32_matrix, const GemmDesc* d_desc, const GemmTask* d_task, int ntask,
                 hipStream_t st) {
  if (ntask <= 0) return;
  if (role == GemmRole::Plan) {
    OSHT_CHECK(!fp32_matrix, OSHT_EINVAL, "plan GEMMs run in FP64");
    launch<true, false, double, RolePlan>(d_desc, d_task, ntask, st);
  } else if (fp32_matrix) {
    launch_role<float>(role, d_desc, d_task, ntask, st);
  } else {
    launch_role<double>(role, d_desc, d_task, ntask, st);
  }
  OSHT_HIP(hipGetLastError());
}

}  // namespace osht
