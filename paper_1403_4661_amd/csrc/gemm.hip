// Batched GEMM on CDNA4 matrix cores for the order-wise applies.
//
// C(M x N) = alpha * A(M x K) * B(K x N) + beta * C, with C and B in FP64
// and A (the plan's matrix: A_m, Q_m or their transposes) in FP64 or FP32.
// Rows [m_lo, M) of C are computed and stored.
//
// One workgroup (4 waves) computes a 64 x 64 tile of C for one descriptor;
// wave w owns rows [16w, 16w+16) and all 64 columns as four 16 x 16 MFMA
// accumulators.  Two tile paths:
//  * streaming (column-major A, row-major B: the applies and the forward's
//    correction): A and B tiles go from global memory straight into LDS
//    with several k-tiles in flight (see gemm_tile_stream);
//  * staged (the plan's Newton-Schulz products and the adjoints, which read
//    A transposed): tiles pass through registers into double-buffered LDS,
//    loads following whichever stride is unit.
// Out-of-range rows, columns and k contribute zero, so any M, N, K >= 0 is
// valid.
//
// FP64: v_mfma_f64_16x16x4f64.  Lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register v of lane l holds
// D[l / 16 + 4 v][l % 16].
// FP32: v_mfma_f32_16x16x4f32 on A (stored FP32) and B rounded to FP32 as it
// is read.  Same operand layout; accumulator register v of lane l holds
// D[4 (l / 16) + v][l % 16].  At most 16 k are accumulated in FP32 by the
// matrix core before the partial sums are added into FP64 accumulators, so
// the FP32 accumulation error is that of a 16-term sum whatever K is.
//
// The precision is chosen per descriptor (GemmDesc::fp32), so one launch
// can mix FP32 and FP64 matrices.  The Role parameter names the kernel
// symbol (inverse apply, forward apply, correction, adjoints, plan
// construction), so that per-kernel profiles separate the launches, and
// selects the streaming tile shape.

#include <type_traits>

#include <hip/hip_ext.h>

#include "common.hpp"

namespace osht {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

struct RolePlan {};
struct RoleApplyInverse {};
struct RoleApplyInverse32 {};
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
template <bool ARF, bool BCF, class T>
__device__ __forceinline__ void gemm_tile(const GemmDesc& d, const GemmTask& t, void* smem) {
  constexpr int P = Pad<T>::v;
  constexpr bool F64 = sizeof(T) == 8;
  typedef T RowA[TM + P];
  typedef T RowB[TN + P];
  RowA(*As)[TK] = reinterpret_cast<RowA(*)[TK]>(smem);                      // [2][TK][TM + P]
  RowB(*Bs)[TK] = reinterpret_cast<RowB(*)[TK]>(static_cast<T*>(smem) + 2 * TK * (TM + P));
  const T* __restrict__ A = static_cast<const T*>(d.A);
  const int m0 = t.mt * TM, n0 = t.nt * TN;
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
      if (row >= d.m_lo && row < d.M && col < d.N) {
        double* cp = d.C + (int64_t)row * d.sCr + (int64_t)col * d.sCc;
        double r = d.alpha * acc[nb][v];
        if (d.beta != 0.0) r += d.beta * (*cp);
        *cp = r;
      }
    }
  }
}

// Streaming variant for column-major A and row-major B: both tiles go from
// global memory straight into LDS (global_load_lds, 16 bytes per lane) with
// NS pipeline stages in flight, so each workgroup keeps NS-1 k-tiles of A
// (the stream that sets the pace) outstanding without spending registers on
// them.  Lanes that fall outside A or B (k >= K, rows >= M, columns >= N)
// load from a zero block, so no tile needs zero-filling.  LDS rows are
// XOR-swizzled by 16 elements per k parity (FP64) or k mod 4 (FP32 A) so
// that the four 16-lane groups of an MFMA operand read hit different banks;
// a 16-byte slot (2 FP64 or 4 FP32 rows) is never split by the swizzle.
__device__ __align__(16) double g_gemm_zero[2];

constexpr int TKS = 16;  // k-tile depth
constexpr int NST = 3;   // pipeline stages

template <class T, int TK = TKS, class TB = double>
struct StreamShape {
  static constexpr int ES = sizeof(T);
  static constexpr int LPC = 64 * ES / 16;        // lanes per A column (32 | 16)
  static constexpr int CPI = 64 / LPC;            // A columns per wave load (2 | 4)
  static constexpr int NIA = TK / CPI;            // wave loads per A tile (8 | 4 at TK = 16)
  static constexpr int EB = sizeof(TB);
  static constexpr int LPR = 64 * EB / 16;        // lanes per B row (32 | 16)
  static constexpr int RPI = 64 / LPR;            // B rows per wave load (2 | 4)
  static constexpr int NIB = TK / RPI;            // wave loads per B tile
  static constexpr int PER_WAVE = (NIA + NIB) / 4;
  // every wave issues PER_WAVE loads per stage (the vmcnt waits count on it)
  static_assert(NIA % 4 == 0 && NIB % 4 == 0, "stream loads must split evenly over the four waves");
  static constexpr int A_BYTES = 64 * TK * ES;
  static constexpr int STAGE = A_BYTES + TK * 64 * EB;
  static __device__ __forceinline__ int aswz(int k) { return ES == 8 ? 16 * (k & 1) : 16 * (k & 3); }
  static __device__ __forceinline__ int bswz(int k) { return EB == 8 ? 16 * (k & 1) : 16 * (k & 3); }
};

template <class T, int TK = TKS, class TB = double>
__device__ __forceinline__ void stream_issue(const GemmDesc& d, const T* __restrict__ A, int m0, int n0, int k0,
                                             char* stage) {
  typedef StreamShape<T, TK, TB> S;
  typedef __attribute__((address_space(3))) void* lds_ptr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // A: column c of the tile holds rows m0..m0+63, row r at position r ^ aswz(k)
#pragma unroll
  for (int i = wave; i < S::NIA; i += 4) {
    const int c = i * S::CPI + lane / S::LPC;
    const int pos = (lane % S::LPC) * (16 / S::ES);  // first row position of this slot
    const int k = k0 + c;
    const int r = m0 + (pos ^ S::aswz(k));
    const void* src = (k < d.K && r < d.M) ? (const void*)(A + r + (int64_t)k * d.sAc) : (const void*)g_gemm_zero;
    __builtin_amdgcn_global_load_lds(src, (lds_ptr)(stage + i * 1024), 16, 0, 0);
  }
  // B: row kk of the tile holds columns n0..n0+63, column j at position j ^ bswz(k)
  char* bst = stage + S::A_BYTES;
  const TB* __restrict__ Bp = reinterpret_cast<const TB*>(d.B);
#pragma unroll
  for (int i = wave; i < S::NIB; i += 4) {
    const int kk = S::RPI * i + lane / S::LPR;
    const int pos = (lane % S::LPR) * (16 / S::EB);
    const int k = k0 + kk;
    const int j = n0 + (pos ^ S::bswz(k));
    const void* src = (k < d.K && j < d.N) ? (const void*)(Bp + (int64_t)k * d.sBr + j) : (const void*)g_gemm_zero;
    __builtin_amdgcn_global_load_lds(src, (lds_ptr)(bst + i * 1024), 16, 0, 0);
  }
}

// waits until at most n (0..31) of this wave's stream loads are outstanding:
// vmcnt in bits 3:0 and 15:14, expcnt (6:4) and lgkmcnt (11:8) at their maxima
template <int N>
__device__ __forceinline__ void wait_vm_c() {
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | 0x0F70);
}
__device__ __forceinline__ void wait_vm(int n) {
  switch (n) {
    case 0: wait_vm_c<0>(); break;
    case 1: wait_vm_c<1>(); break;
    case 2: wait_vm_c<2>(); break;
    case 3: wait_vm_c<3>(); break;
    case 4: wait_vm_c<4>(); break;
    case 6: wait_vm_c<6>(); break;
    case 8: wait_vm_c<8>(); break;
    case 9: wait_vm_c<9>(); break;
    case 12: wait_vm_c<12>(); break;
    case 16: wait_vm_c<16>(); break;
    case 18: wait_vm_c<18>(); break;
    case 24: wait_vm_c<24>(); break;
    default: wait_vm_c<0>(); break;
  }
}

// PREFC: C is read (beta != 0) into registers before the k loop, so that its
// latency overlaps the streaming instead of following it (the forward's
// correction, whose k depth is at most one block of levels).
// W22: the four waves cover the 64x64 tile as 2x2 blocks of 32x32 (each
// 2x2 MFMA tiles of 16x16) instead of four 16x64 strips, so a wave reads two
// A and two B operands from LDS per four MFMAs instead of one A and four B.
template <class T, int TK = TKS, int NS = NST, class TB = double, bool PREFC = false, bool W22 = false>
__device__ __forceinline__ void gemm_tile_stream(const GemmDesc& d, const GemmTask& t, char* smem) {
  typedef StreamShape<T, TK, TB> S;
  constexpr bool F64 = sizeof(T) == 8;
  const T* __restrict__ A = static_cast<const T*>(d.A);
  const int m0 = t.mt * TM, n0 = t.nt * TN;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, li = lane & 15;
  // first row / column (within the tile) of MFMA tile nb of this wave
  auto rowb = [&](int nb) { return W22 ? (wave & 1) * 32 + (nb >> 1) * 16 : wave * 16; };
  auto colb = [&](int nb) { return W22 ? (wave >> 1) * 32 + (nb & 1) * 16 : nb * 16; };
  dbl4 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = dbl4{0.0, 0.0, 0.0, 0.0};
  double cpre[4][4];
  if constexpr (PREFC) {
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = m0 + rowb(nb) + (F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
        const int col = n0 + colb(nb) + (lane & 15);
        cpre[nb][v] = (d.beta != 0.0 && r >= d.m_lo && r < d.M && col < d.N)
                          ? d.C[(int64_t)r * d.sCr + (int64_t)col * d.sCc]
                          : 0.0;
      }
    }
  }
  const int nt = (d.K + TK - 1) / TK;
#pragma unroll
  for (int st = 0; st < NS - 1; ++st)
    if (st < nt) stream_issue<T, TK, TB>(d, A, m0, n0, st * TK, smem + st * S::STAGE);
  for (int kt = 0; kt < nt; ++kt) {
    // tiles issued after kt: min(NS-2, nt-1-kt) before this iteration's issue
    const int ahead = min(NS - 2, nt - 1 - kt);
    wait_vm(ahead * S::PER_WAVE);
    // tile kt complete in LDS, tile kt-1's stage free.  A bare barrier: a
    // fence here would also wait for the loads still in flight.
    __builtin_amdgcn_s_barrier();
    if (kt + NS - 1 < nt)
      stream_issue<T, TK, TB>(d, A, m0, n0, (kt + NS - 1) * TK, smem + ((kt + NS - 1) % NS) * S::STAGE);
    const char* stage = smem + (kt % NS) * S::STAGE;
    const T* As = reinterpret_cast<const T*>(stage);
    const TB* Bs = reinterpret_cast<const TB*>(stage + S::A_BYTES);
    if constexpr (F64 && W22) {
#pragma unroll
      for (int s = 0; s < TK / 4; ++s) {
        const int k = 4 * s + kq;
        double a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[i] = As[k * 64 + ((rowb(2 * i) + li) ^ S::aswz(k))];
          b[i] = Bs[k * 64 + ((colb(i) + li) ^ S::bswz(k))];
        }
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
          acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[nb >> 1], b[nb & 1], acc[nb], 0, 0, 0);
      }
    } else if constexpr (F64) {
#pragma unroll
      for (int s = 0; s < TK / 4; ++s) {
        const int k = 4 * s + kq;
        const double a = As[k * 64 + ((wave * 16 + li) ^ S::aswz(k))];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const double b = Bs[k * 64 + ((nb * 16 + li) ^ S::bswz(k))];
          acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[nb], 0, 0, 0);
        }
      }
    } else {
      flt4 c[4];
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) c[nb] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < TK / 4; ++s) {
        const int k = 4 * s + kq;
        if constexpr (W22) {
          float a[2], b[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            a[i] = As[k * 64 + ((rowb(2 * i) + li) ^ S::aswz(k))];
            b[i] = (float)Bs[k * 64 + ((colb(i) + li) ^ S::bswz(k))];
          }
#pragma unroll
          for (int nb = 0; nb < 4; ++nb)
            c[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[nb >> 1], b[nb & 1], c[nb], 0, 0, 0);
        } else {
          const float a = As[k * 64 + ((wave * 16 + li) ^ S::aswz(k))];
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) {
            const float b = (float)Bs[k * 64 + ((nb * 16 + li) ^ S::bswz(k))];
            c[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[nb], 0, 0, 0);
          }
        }
        if (TK > 16 && s % 4 == 3 && s + 1 < TK / 4) {  // FP32 partial sums cover 16 k at most
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[nb][v] += (double)c[nb][v];
            c[nb] = flt4{0.f, 0.f, 0.f, 0.f};
          }
        }
      }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[nb][v] += (double)c[nb][v];
    }
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = m0 + rowb(nb) + (F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
      const int col = n0 + colb(nb) + (lane & 15);
      if (r >= d.m_lo && r < d.M && col < d.N) {
        const int64_t ci = (int64_t)r * d.sCr + (int64_t)col * d.sCc;
        if constexpr (std::is_same<TB, float>::value) {  // FP32 inverse apply: C may be FP32
          if (d.c32) {
            reinterpret_cast<float*>(d.C)[ci] = (float)(d.alpha * acc[nb][v]);
            continue;
          }
        }
        double* cp = d.C + ci;
        double x = d.alpha * acc[nb][v];
        if (d.beta != 0.0) x += d.beta * (PREFC ? cpre[nb][v] : *cp);
        *cp = x;
      }
    }
  }
}

// LDS of one tile pair: the FP64 layout is the larger one.
constexpr int kSmemDoubles = 2 * 2 * TK * (TM + Pad<double>::v);
static_assert(2 * TK * (TM + Pad<float>::v) * 2 * sizeof(float) <= kSmemDoubles * sizeof(double), "LDS size");

// Default stream shape (k depth, stages), measured on MI355X.  FP64 tiles
// run 16 deep in 2 stages (32 KB of LDS): in the forward's per-block
// launches so that four workgroups fit a CU (three 48 KB stages allowed three
// and the step was 0.03-0.09 ms slower), in the FP64 inverse apply 1.41 ->
// 1.24 ms against 32-deep tiles (64 KB, two per CU).  Tiles with an FP32 A
// and FP64 B (NS32) run in 2 stages too (24 KB; 3 stages, 36 KB, were
// slightly slower), so the forward blocks take 32 KB.  The FP32 inverse apply runs
// 16-deep tiles in 2 stages (16 KB): 0.76 -> 0.74 ms against 32-deep ones;
// 3 stages of 32 or of 16 were slower.
//
// Stream shapes of the streaming roles (k depth TK, stages NS for FP64 A
// and NS32 for FP32 A), V = 0 the default and 1, 2 the alternatives that the
// plan-time tuner (OSHT_TUNE) also times for the inverse and forward
// applies.  Every shape sums k in the same order (FP64: one MFMA k-step of
// 4 after another; FP32 A: partial sums over 16 k added into FP64), so the
// shapes give bit-identical results.
template <int V> struct StreamVar;
template <> struct StreamVar<0> { static constexpr int TK = 16, NS = 2, NS32 = 2; };
template <> struct StreamVar<1> { static constexpr int TK = 16, NS = 3, NS32 = 3; };
template <> struct StreamVar<2> { static constexpr int TK = 32, NS = 2, NS32 = 2; };
template <class Role, int V> struct StreamCfg : StreamVar<V> {
  static constexpr bool W22 = true;
};

// Each task's descriptor selects the matrix precision (GemmDesc::fp32).
template <bool ARF, bool BCF, class Role, int V>
__global__ __launch_bounds__(256) void gemm_kernel(const GemmDesc* __restrict__ descs,
                                                   const GemmTask* __restrict__ tasks) {
  typedef StreamCfg<Role, V> SC;
  constexpr bool kF32 = std::is_same<Role, RoleApplyInverse32>::value;
  constexpr int kStream64 = SC::NS * StreamShape<double, SC::TK>::STAGE / 8;
  constexpr int kStream32 = SC::NS32 * StreamShape<float, SC::TK, double>::STAGE / 8;
  constexpr int kStream = kF32 ? SC::NS * StreamShape<float, SC::TK, float>::STAGE / 8
                               : (kStream64 > kStream32 ? kStream64 : kStream32);
  __shared__ __align__(16) double smem[kF32 ? kStream
                                             : (ARF && BCF) ? (kStream > kSmemDoubles ? kStream : kSmemDoubles)
                                                            : kSmemDoubles];
  // Workgroups are dispatched round-robin over the 8 XCDs.  Tasks come in
  // descriptor order, the M tiles of one descriptor (which share its B panel)
  // adjacent; runs of 16 consecutive tasks go to workgroups of one XCD, so a
  // panel is fetched into one L2, while successive runs rotate over the XCDs
  // (descriptors of very different sizes stay balanced).  Bijective on
  // [0, gridDim.x); the tail round uses the plain block split.
  constexpr int C = 16, RND = 8 * C;
  const int G = gridDim.x, b = blockIdx.x, base = (b / RND) * RND, p = b - base;
  int ti;
  if (base + RND <= G) {
    ti = base + (p & 7) * C + (p >> 3);
  } else {
    const int S = G - base, q = S >> 3, r = S & 7, x = p & 7, l = p >> 3;
    ti = base + (x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l);
  }
  const GemmTask t = tasks[ti];
  const GemmDesc d = descs[t.desc];
  // column-major A streams through LDS
  if constexpr (kF32) {
    gemm_tile_stream<float, SC::TK, SC::NS, float, false, SC::W22>(d, t, reinterpret_cast<char*>(smem));
  } else if constexpr (ARF && BCF) {
    constexpr bool kPrefC = std::is_same<Role, RoleCorrection>::value;
    if (d.fp32) gemm_tile_stream<float, SC::TK, SC::NS32, double, kPrefC, SC::W22>(d, t, reinterpret_cast<char*>(smem));
    else gemm_tile_stream<double, SC::TK, SC::NS, double, kPrefC, SC::W22>(d, t, reinterpret_cast<char*>(smem));
  } else {
    if (d.fp32) gemm_tile<ARF, BCF, float>(d, t, smem);
    else gemm_tile<ARF, BCF, double>(d, t, smem);
  }
}

// With events, they take the dispatch's own start and end timestamps
// (hipExtLaunchKernel), so timing adds no packets between launches.
template <bool ARF, bool BCF, class Role, int V>
void launch(const GemmDesc* d_desc, const GemmTask* d_task, int ntask, hipStream_t st, hipEvent_t e0,
            hipEvent_t e1) {
  if (e0) {
    void* args[] = {(void*)&d_desc, (void*)&d_task};
    OSHT_HIP(hipExtLaunchKernel((const void*)gemm_kernel<ARF, BCF, Role, V>, dim3(ntask), dim3(256), args, 0, st, e0,
                                e1, 0));
  } else {
    hipLaunchKernelGGL((gemm_kernel<ARF, BCF, Role, V>), dim3(ntask), dim3(256), 0, st, d_desc, d_task);
  }
}

template <class Role>
void launch_var(int var, const GemmDesc* d_desc, const GemmTask* d_task, int ntask, hipStream_t st, hipEvent_t e0,
                hipEvent_t e1) {
  switch (var) {
    case 1: launch<true, true, Role, 1>(d_desc, d_task, ntask, st, e0, e1); break;
    case 2: launch<true, true, Role, 2>(d_desc, d_task, ntask, st, e0, e1); break;
    default: launch<true, true, Role, 0>(d_desc, d_task, ntask, st, e0, e1); break;
  }
}

}  // namespace

void gemm_tasks(const std::vector<GemmDesc>& descs, std::vector<GemmTask>& tasks) {
  tasks.clear();
  for (size_t i = 0; i < descs.size(); ++i) {
    const int mt = (int)ceil_div(descs[i].M, TM), nt = (int)ceil_div(descs[i].N, TN);
    for (int a = descs[i].m_lo / TM; a < mt; ++a)
      for (int b = 0; b < nt; ++b) tasks.push_back(GemmTask{(int32_t)i, a, b, 0});
  }
}

void launch_gemm(GemmRole role, const GemmDesc* d_desc, const GemmTask* d_task, int ntask, hipStream_t st,
                 hipEvent_t e0, hipEvent_t e1, int var) {
  if (ntask <= 0) return;
  switch (role) {
    case GemmRole::Plan: launch<true, false, RolePlan, 0>(d_desc, d_task, ntask, st, e0, e1); break;
    case GemmRole::ApplyInverse: launch_var<RoleApplyInverse>(var, d_desc, d_task, ntask, st, e0, e1); break;
    case GemmRole::ApplyInverse32: launch_var<RoleApplyInverse32>(var, d_desc, d_task, ntask, st, e0, e1); break;
    case GemmRole::ApplyForward: launch_var<RoleApplyForward>(var, d_desc, d_task, ntask, st, e0, e1); break;
    case GemmRole::Correction: launch<true, true, RoleCorrection, 0>(d_desc, d_task, ntask, st, e0, e1); break;
    case GemmRole::Adjoint: launch<false, true, RoleAdjoint, 0>(d_desc, d_task, ntask, st, e0, e1); break;
  }
  OSHT_HIP(hipGetLastError());
}

}  // namespace osht
