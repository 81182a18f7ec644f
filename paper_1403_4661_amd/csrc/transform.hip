// The four transforms: inverse (Procedure 2), forward (Procedure 1) and
// their adjoints, as sequences of gather / order-wise GEMM / scatter / ring
// DFT kernels on one stream.
//
// Internal per-call buffers (doubles, map-fastest so that GEMM operands are
// contiguous):
//   X[slot][row][col], Y[slot][row][col]  row < L, col < ncols
//   H[(k^2 + q) * B + b]                   ring bins (complex)
// Column col of a slot encodes (sign, map, re/im): spin 0 uses
// col = sgn * 2B + 2b + part for the orders +am (sgn 0) and -am (sgn 1);
// spin s != 0 uses col = 2b + part for the slot's single order.
//
// Inverse:  X_m = coefficients of order m (rows l = l0..L-1)
//           Y_m = A_m X_m : G'_m(theta_k) on every ring k
//           f   = per ring, fold order m into bin (m mod n_k), inverse DFT.
// Forward (descending |m|):
//           X_m[k - |m|] = H_k[m mod n_k] - sum_{m' = m mod n_k, |m'| > k} G'_{m'}(theta_k)
//           Y_m = Q_m X_m = [ f_m ; G'_m(theta_k), k < |m| ]
// The aliases G'_{m'}(theta_k) of the already-solved orders are read back
// from the Y blocks of those orders (their bottom |m'| rows), so no bin is
// ever updated in place and every sum is taken in a fixed order.
// Spin 0: P_{-m} = (-1)^m P_m, hence Q_{-m} = [(-1)^m P_m^{-1}; A^top_m P_m^{-1}]
// and A_{-m} = (-1)^m A_m; the sign is applied where coefficients enter or
// leave the slot buffers.

#include "xform.hpp"

namespace osht {

void launch_fold(const Plan& p, const double* Y, double* H, int64_t B, hipStream_t st);
void launch_ring_synthesis(const Plan& p, const double* H, int scale_inv_n, double* f, int64_t B, hipStream_t st,
                           int64_t real_maps = 0);

namespace {

// Coefficients (l-major, map-major) <-> slot layout, through an LDS tile of
// 64 consecutive orders x 16 maps per step: one workgroup per (degree l,
// chunk of 64 orders), so that the long rows of high degrees are spread.
// The grid holds only the chunks that exist (degree l has floor(l/32) + 1);
// with a (chunk, degree) rectangle half of the workgroups returned at once,
// and both transposes took 0.26 instead of 0.21 ms at L = 1024, B = 16.
// to_slots: X[slot(m)][l - l0(m)][col(m, b)] = sign(m) * flm[b][l^2 + l + m]
// else:     flm[b][l^2 + l + m] = sign(m) * Y[slot(m)][l - l0(m)][col(m, b)],
//           zero when l < l0(m) (spin: degrees below |s|).
// sign(m) = (-1)^|m| for spin 0 and m < 0 (both orders share A_|m|, Q_|m|).
// With TO_SLOTS the slot values are written as O (double2, or float2 for
// the FP32 inverse apply, which rounds its right-hand side to FP32).
// Workgroups before degree l: sum over l' < l of the floor(l'/32) + 1 chunks
// of 64 orders that degree l' has.
__device__ __forceinline__ int chunks_before(int l) {
  const int q = l >> 5, r = l & 31;
  return l + 16 * q * (q - 1) + q * r;
}

template <bool TO_SLOTS, class O = double2>
__global__ __launch_bounds__(256) void coef_transpose_kernel(Geo g, const double2* __restrict__ src,
                                                             O* __restrict__ dst) {
  __shared__ double2 tile[16][65];
  // one workgroup per (degree, chunk of 64 orders): find the degree
  const int bid = blockIdx.x;
  int lo = 0, hi = g.L;  // chunks_before(lo) <= bid < chunks_before(hi)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (chunks_before(mid) <= bid) lo = mid;
    else hi = mid;
  }
  const int l = lo;
  const int nc = g.ncols >> 1;
  const int as = g.s < 0 ? -g.s : g.s;
  const int64_t LL = (int64_t)g.L * g.L;
  {
    const int m0 = -l + 64 * (bid - chunks_before(l));
    const int nm = min(64, l - m0 + 1);
    for (int b0 = 0; b0 < g.B; b0 += 16) {
      const int nb = min(16, g.B - b0);
      if constexpr (TO_SLOTS) {
        for (int e = threadIdx.x; e < nb * nm; e += blockDim.x) {
          const int bb = e / nm, mi = e - bb * nm;
          tile[bb][mi] = src[(int64_t)(b0 + bb) * LL + (int64_t)l * l + l + m0 + mi];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nm * nb; e += blockDim.x) {
          const int mi = e / nb, bb = e - mi * nb;
          const int m = m0 + mi, am = m < 0 ? -m : m;
          const int l0 = am > as ? am : as;
          if (l < l0) continue;
          const int slot = g.s == 0 ? am : m + g.L - 1;
          const int sgn = (g.s == 0 && m < 0) ? 1 : 0;
          double2 v = tile[bb][mi];
          if (sgn && (am & 1)) { v.x = -v.x; v.y = -v.y; }
          O o;
          o.x = v.x;
          o.y = v.y;
          dst[((int64_t)slot * g.L + (l - l0)) * nc + sgn * g.B + b0 + bb] = o;
        }
      } else {
        for (int e = threadIdx.x; e < nm * nb; e += blockDim.x) {
          const int mi = e / nb, bb = e - mi * nb;
          const int m = m0 + mi, am = m < 0 ? -m : m;
          const int l0 = am > as ? am : as;
          double2 v = {0.0, 0.0};
          if (l >= l0) {
            const int slot = g.s == 0 ? am : m + g.L - 1;
            const int sgn = (g.s == 0 && m < 0) ? 1 : 0;
            v = src[((int64_t)slot * g.L + (l - l0)) * nc + sgn * g.B + b0 + bb];
            if (sgn && (am & 1)) { v.x = -v.x; v.y = -v.y; }
          }
          tile[bb][mi] = v;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nb * nm; e += blockDim.x) {
          const int bb = e / nm, mi = e - bb * nm;
          dst[(int64_t)(b0 + bb) * LL + (int64_t)l * l + l + m0 + mi] = tile[bb][mi];
        }
      }
      __syncthreads();
    }
  }
}

// Forward, one level: X[slot][r][col], ring k = |m| + r: bin minus aliases.
__global__ __launch_bounds__(256) void fwd_gather_kernel(Geo g, const Slot* __restrict__ slots, int slot0,
                                                         const double* __restrict__ H, const double* __restrict__ Y,
                                                         double* __restrict__ X) {
  const int slot = slot0 + blockIdx.y;
  const Slot sl = slots[slot];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = e / g.ncols, col = e % g.ncols;
  if (r >= sl.R) return;
  int sgn, b, part, m;
  decode_col(g, sl, col, sgn, b, part, m);
  const int am = m < 0 ? -m : m;
  const int k = am + r, n = 2 * k + 1;
  const int bin = pmod(m, n);
  double v = H[(((int64_t)k * k + bin) * g.B + b) * 2 + part];
  const int start = bin - ((bin + g.L - 1) / n) * n;  // smallest m' >= -(L-1), m' = m (mod n)
  for (int mp = start; mp <= g.L - 1; mp += n) {
    if (mp == m) continue;
    v -= Y[alias_index(g, slots, mp, k, b, part)];
  }
  X[((int64_t)slot * g.L + r) * g.ncols + col] = v;
}

// Inverse adjoint: X[slot][k][col] = Hbar_k[m mod n_k] for every ring k.
__global__ __launch_bounds__(256) void iadj_gather_kernel(Geo g, const Slot* __restrict__ slots, int slot0,
                                                          const double* __restrict__ H, double* __restrict__ X) {
  const int slot = slot0 + blockIdx.y;
  const Slot sl = slots[slot];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = e / g.ncols, col = e % g.ncols;
  if (k >= g.L) return;
  int sgn, b, part, m;
  decode_col(g, sl, col, sgn, b, part, m);
  const int n = 2 * k + 1;
  X[((int64_t)slot * g.L + k) * g.ncols + col] = H[(((int64_t)k * k + pmod(m, n)) * g.B + b) * 2 + part];
}

// Forward adjoint, one level: X[slot][i][col] = [ ybar (i < K) ; -Hbar_k[m mod n_k] (k = i - K < |m|) ].
__global__ __launch_bounds__(256) void fadj_gather_kernel(Geo g, const Slot* __restrict__ slots, int slot0,
                                                          const double* __restrict__ flmbar, const double* __restrict__ H,
                                                          double* __restrict__ X) {
  const int slot = slot0 + blockIdx.y;
  const Slot sl = slots[slot];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = e / g.ncols, col = e % g.ncols;
  int sgn, b, part, m;
  decode_col(g, sl, col, sgn, b, part, m);
  const int am = m < 0 ? -m : m;
  if (i >= sl.K + am) return;
  double v;
  if (i < sl.K) {
    const int l = sl.l0 + i;
    v = flmbar[((int64_t)b * g.L * g.L + (int64_t)l * l + l + m) * 2 + part];
    if (g.s == 0 && sgn && (am & 1)) v = -v;
  } else {
    const int k = i - sl.K, n = 2 * k + 1;
    v = -H[(((int64_t)k * k + pmod(m, n)) * g.B + b) * 2 + part];
  }
  X[((int64_t)slot * g.L + i) * g.ncols + col] = v;
}

// Forward adjoint, one level: Hbar_k[m mod n_k] = Y[slot][k - |m|][col], k >= |m|.
__global__ __launch_bounds__(256) void fadj_scatter_kernel(Geo g, const Slot* __restrict__ slots, int slot0,
                                                           const double* __restrict__ Y, double* __restrict__ H) {
  const int slot = slot0 + blockIdx.y;
  const Slot sl = slots[slot];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = e / g.ncols, col = e % g.ncols;
  if (r >= sl.R) return;
  int sgn, b, part, m;
  decode_col(g, sl, col, sgn, b, part, m);
  if (g.s == 0 && sgn && sl.m == 0) return;  // -0 duplicates +0
  const int am = m < 0 ? -m : m;
  const int k = am + r, n = 2 * k + 1;
  H[(((int64_t)k * k + pmod(m, n)) * g.B + b) * 2 + part] = Y[((int64_t)slot * g.L + r) * g.ncols + col];
}


}  // namespace

// ---------------------------------------------------------------- host side
const char* const kApplyName[kNumDir] = {"apply_inverse",           "apply_forward",
                                         "apply_inverse_adjoint",   "apply_forward_adjoint",
                                         "apply_forward_correction", "apply_forward",
                                         "apply_forward_correction", "apply_forward_adjoint_correction"};

// Workspace for batch B (grown on demand, never shrunk) and the GEMM
// descriptor tables of B.  Tables are kept per batch size for the current
// workspace, so that alternating batch sizes neither synchronise the device
// nor rewrite tables that earlier, still running work may read; only a
// workspace growth or an eviction (more than kMaxTables batch sizes) waits
// for the device.
void ensure_workspace(Plan& p, int64_t B) {
  const int64_t ncols = p.ncols_per_map * B;
  const size_t xy = sizeof(double) * (size_t)p.nslots * p.L * ncols;
  const size_t hb = sizeof(double) * 2 * (size_t)p.L * p.L * B;
  const size_t db = sizeof(double) * (size_t)p.nslots * std::max(p.fb.b, 1) * ncols;
  // int8-digit plans: digit planes and exponents of the right-hand sides
  const size_t x8 = p.oz ? (size_t)p.nslots * p.oz * oz_x_cols(p, B) * (size_t)oz_x_ld(p) : 0;
  const size_t xe = p.oz ? sizeof(int32_t) * (size_t)p.nslots * oz_x_cols(p, B) : 0;
  const bool grow = (xy > p.w_X.bytes) || (hb > p.w_H.bytes) || (db > p.w_D.bytes) || (x8 > p.w_X8.bytes) ||
                    (xe > p.w_Xexp.bytes);
  if (grow) {
    // the buffers and every table pointing into them are replaced: earlier
    // work on any stream may still use them
    OSHT_HIP(hipDeviceSynchronize());
    p.tabs.clear();
    p.tab = nullptr;
    ++p.ws_version;
    p.w_X.reserve(xy);
    p.w_Y.reserve(xy);
    p.w_H.reserve(hb);
    p.w_D.reserve(db);
    p.w_X8.reserve(x8);
    p.w_Xexp.reserve(xe);
  }
  for (size_t i = 0; i < p.tabs.size(); ++i) {
    if (p.tabs[i]->B == B) {
      std::unique_ptr<DescTables> t = std::move(p.tabs[i]);  // most recently used last
      p.tabs.erase(p.tabs.begin() + (long)i);
      p.tabs.push_back(std::move(t));
      p.tab = p.tabs.back().get();
      return;
    }
  }
  if ((int)p.tabs.size() >= Plan::kMaxTables) {
    OSHT_HIP(hipDeviceSynchronize());
    p.tabs.erase(p.tabs.begin());
    ++p.ws_version;
  }
  p.tabs.push_back(std::unique_ptr<DescTables>(new DescTables));
  DescTables& t = *p.tabs.back();
  p.tab = &t;
  t.B = B;
  double* X = p.w_X.as<double>();
  double* Y = p.w_Y.as<double>();
  double* D = p.w_D.as<double>();
  // Matrix element offsets are the same in the FP64 and FP32 copies.  FP32
  // plans apply A_m (inverse and its adjoint) in FP32; OSHT_PREC_FP32_FWD
  // also the coefficient rows of Q_m (P_m^{-1}).  The alias rows of Q_m
  // (A_m^top P_m^{-1}), which feed the descending-order chain, and the
  // forward adjoint stay FP64.
  const double* A64 = p.d_A.as<double>();
  const double* Q64 = p.d_Q.as<double>();
  const float* A32 = p.d_A32.as<float>();
  const float* Q32 = p.d_Q32.as<float>();
  const bool f32 = p.fp32;          // A_m in FP32
  const bool f32q = p.fp32_fwd;     // coefficient rows of Q_m in FP32
  const int bD = std::max(p.fb.b, 1);
  std::vector<int32_t> wcorr(p.nslots, 0), q0of(p.nslots, 0);  // correction width, block start per slot
  for (size_t blk = 0; blk + 1 < p.fb.slot_ptr.size(); ++blk)
    for (int i = p.fb.slot_ptr[blk]; i < p.fb.slot_ptr[blk + 1]; ++i) {
      const int slot = p.fb.slot_list[i];
      wcorr[slot] = p.fb.q1[blk] - std::abs(p.slots[slot].m);
      q0of[slot] = p.fb.q0[blk];
    }
  for (int dir = 0; dir < kNumDir; ++dir) {
    for (int i = 0; i < p.nslots; ++i) {
      const Slot& sl = p.slots[i];
      const int am = std::abs(sl.m);
      double* Xs = X + (int64_t)i * p.L * ncols;
      double* Ys = Y + (int64_t)i * p.L * ncols;
      GemmDesc d{};
      d.B = Xs; d.sBr = ncols; d.sBc = 1;
      d.C = Ys; d.sCr = ncols; d.sCc = 1;
      d.N = (int)ncols; d.alpha = 1.0; d.beta = 0.0;
      auto setA = [&](bool use32, bool isA, int64_t off) {
        d.fp32 = use32 ? 1 : 0;
        if (use32) d.A = (isA ? A32 : Q32) + off;
        else d.A = (isA ? A64 : Q64) + off;
      };
      if (dir == kInv) {
        setA(f32, true, sl.offA); d.sAr = 1; d.sAc = sl.ldA; d.M = p.L; d.K = sl.K;
        if (f32) {  // right-hand side and output in FP32, in the same workspaces
          d.B = reinterpret_cast<const double*>(reinterpret_cast<const float*>(X) + (int64_t)i * p.L * ncols);
          d.b32 = 1;
          d.C = reinterpret_cast<double*>(reinterpret_cast<float*>(Y) + (int64_t)i * p.L * ncols);
          d.c32 = 1;
        }
      }
      if (dir == kIadj) { setA(f32, true, sl.offA); d.sAr = sl.ldA; d.sAc = 1; d.M = sl.K; d.K = p.L; }
      if (dir == kFadj) { setA(false, false, sl.offQ); d.sAr = sl.ldQ; d.sAc = 1; d.M = sl.R; d.K = sl.K + am; }
      if (dir == kFadjCorr) {  // Z -= Q^T[:, K + q0 .. K + |m|) E, E rows k - q0
        setA(false, false, sl.offQ + sl.K + q0of[i]);
        d.sAr = sl.ldQ; d.sAc = 1; d.M = sl.R; d.K = std::max(0, am - q0of[i]);
        d.B = D + (int64_t)i * bD * ncols;
        d.alpha = -1.0; d.beta = 1.0;
      }
      if (dir == kFwd || dir == kCorr || dir == kFwdAlias || dir == kCorrAlias) {
        // With FP32 coefficient rows: the 64-row tiles that hold only
        // coefficient rows, [0, Kc) with Kc = 64 floor(K / 64), in the main
        // descriptor (FP32), the rest [Kc, K + |m|) -- the tile straddling
        // the coefficient/alias boundary and the alias rows -- in the alias
        // one (FP64), so that every 64-row tile is computed once.  Otherwise
        // all rows in the main descriptor.  Descriptors keep column-base
        // pointers and select rows by [m_lo, M).
        const bool alias = dir == kFwdAlias || dir == kCorrAlias;
        const int Kc = sl.K / 64 * 64;
        const int r0 = alias ? Kc : 0;
        const int r1 = f32q ? (alias ? sl.K + am : Kc) : (alias ? 0 : sl.K + am);
        setA(f32q && !alias, false, sl.offQ);
        d.sAr = 1; d.sAc = sl.ldQ;
        d.m_lo = r1 > r0 ? r0 : 0;
        d.M = r1 > r0 ? r1 : 0;
        d.K = sl.R;
        if (dir == kCorr || dir == kCorrAlias) {  // Y -= Q[:, 0:w] D
          d.K = std::min(wcorr[i], sl.R);
          d.B = D + (int64_t)i * bD * ncols;
          d.alpha = -1.0; d.beta = 1.0;
        }
      }
      t.h_gdesc.push_back(d);
    }
  }
  gemm_tasks(t.h_gdesc, t.h_gtask);
  upload(t.d_gdesc, t.h_gdesc);
  upload(t.d_gtask, t.h_gtask);
  if (p.oz) {
    oz_descs(p, B, Y, p.w_X8.as<int8_t>(), p.w_Xexp.as<int32_t>(), t.h_oz, t.h_oztask);
    upload(t.d_ozdesc, t.h_oz);
    upload(t.d_oztask, t.h_oztask);
  }
  // per-block task lists of the blocked forward: [Q apply, correction]
  std::vector<GemmTask> bt;
  t.h_btask_ptr.clear();
  const int nblk = (int)p.fb.q0.size();
  auto emit = [&](int d) {
    const GemmDesc& g = t.h_gdesc[d];
    if (g.K <= 0 || g.M <= g.m_lo) return;
    for (int a = g.m_lo / 64; a < (int)ceil_div(g.M, 64); ++a)
      for (int c = 0; c < (int)ceil_div(g.N, 64); ++c) bt.push_back(GemmTask{d, a, c, 0});
  };
  for (int blk = 0; blk < nblk; ++blk) {
    const bool has_unk = p.fb.unk_ptr[blk + 1] > p.fb.unk_ptr[blk];
    t.h_btask_ptr.push_back((int32_t)bt.size());
    for (int dir : {kFwd, kFwdAlias})
      for (int i = p.fb.slot_ptr[blk]; i < p.fb.slot_ptr[blk + 1]; ++i) emit(dir * p.nslots + p.fb.slot_list[i]);
    t.h_btask_ptr.push_back((int32_t)bt.size());
    if (has_unk)
      for (int dir : {kCorr, kCorrAlias})
        for (int i = p.fb.slot_ptr[blk]; i < p.fb.slot_ptr[blk + 1]; ++i) emit(dir * p.nslots + p.fb.slot_list[i]);
  }
  t.h_btask_ptr.push_back((int32_t)bt.size());
  upload(t.d_btask, bt);
  // per-block task lists of the blocked forward adjoint: [Q^T apply, correction]
  std::vector<GemmTask> at;
  t.h_atask_ptr.clear();
  auto emit_to = [&](std::vector<GemmTask>& v, int d) {
    const GemmDesc& g = t.h_gdesc[d];
    if (g.K <= 0 || g.M <= g.m_lo) return;
    for (int a = g.m_lo / 64; a < (int)ceil_div(g.M, 64); ++a)
      for (int c = 0; c < (int)ceil_div(g.N, 64); ++c) v.push_back(GemmTask{d, a, c, 0});
  };
  for (int blk = 0; blk < nblk; ++blk) {
    const bool has_unk = p.fb.unk_ptr[blk + 1] > p.fb.unk_ptr[blk];
    t.h_atask_ptr.push_back((int32_t)at.size());
    for (int i = p.fb.slot_ptr[blk]; i < p.fb.slot_ptr[blk + 1]; ++i) emit_to(at, kFadj * p.nslots + p.fb.slot_list[i]);
    t.h_atask_ptr.push_back((int32_t)at.size());
    if (has_unk)
      for (int i = p.fb.slot_ptr[blk]; i < p.fb.slot_ptr[blk + 1]; ++i)
        emit_to(at, kFadjCorr * p.nslots + p.fb.slot_list[i]);
  }
  t.h_atask_ptr.push_back((int32_t)at.size());
  upload(t.d_atask, at);
}

void prepare_transforms(Plan& p, int64_t B) { ensure_workspace(p, B); }

void invalidate_tables(Plan& p) {
  if (p.tabs.empty()) return;
  OSHT_HIP(hipDeviceSynchronize());
  p.tabs.clear();
  p.tab = nullptr;
  ++p.ws_version;
}

namespace {

// Real maps (spin 0): complex map j carries real maps 2j and 2j+1 as
// z = S(a) + i S(b), S(x)_lm = (x_lm + (-1)^m conj(x_{l,-m})) / 2 (Eq.
// yellm:conj; the inverse of S(x) is the real part of the inverse of x).  In
// the slot row (l, |m|) of map j, P = z_{l,|m|} sits in the +m columns and
// N = (-1)^m z_{l,-|m|} in the -m columns, so with alpha = S(a)_{l,|m|} and
// beta = S(b)_{l,|m|}:  P = alpha + i beta,  N = conj(alpha) + i conj(beta);
// and back:  a_{l,|m|} = (P + conj N)/2,  a_{l,-|m|} = (-1)^m (N + conj P)/2,
// b_{l,|m|} = (P - conj N)/(2i),  b_{l,-|m|} = (-1)^m (N - conj P)/(2i).
// One workgroup per (degree l, 64 orders |m|), 8 complex maps per LDS step.
// Order 0 has only the +m columns (its -m columns are not read).
template <class O>
__global__ __launch_bounds__(256) void real_coef_to_slots_kernel(Geo g, int Breal, const double2* __restrict__ flm,
                                                                 O* __restrict__ X) {
  __shared__ double2 ta[2][16][65];  // [sign][real map in chunk][order in chunk]
  const int l = blockIdx.y, am0 = 64 * (int)blockIdx.x;
  if (am0 > l) return;  // uniform over the workgroup
  const int nam = min(64, l - am0 + 1);
  const int nc = g.ncols >> 1;
  const int64_t LL = (int64_t)g.L * g.L;
  for (int j0 = 0; j0 < g.B; j0 += 8) {
    const int nj = min(8, g.B - j0);
    for (int e = threadIdx.x; e < 2 * 2 * nj * nam; e += blockDim.x) {
      const int ai = e % nam, rest = e / nam;
      const int rr = rest % (2 * nj), sg = rest / (2 * nj);
      const int r = 2 * j0 + rr, m = sg ? -(am0 + ai) : am0 + ai;
      ta[sg][rr][ai] = r < Breal ? flm[(int64_t)r * LL + (int64_t)l * l + l + m] : double2{0.0, 0.0};
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nam * 2 * nj; e += blockDim.x) {
      const int col = e % (2 * nj), ai = e / (2 * nj);
      const int sg = col / nj, jj = col - sg * nj;
      const int am = am0 + ai;
      if (am == 0 && sg) continue;
      const double s = (am & 1) ? -1.0 : 1.0;
      const double2 ap = ta[0][2 * jj][ai], an = ta[1][2 * jj][ai];
      const double2 bp = ta[0][2 * jj + 1][ai], bn = ta[1][2 * jj + 1][ai];
      const double2 al = {0.5 * (ap.x + s * an.x), 0.5 * (ap.y - s * an.y)};
      const double2 be = {0.5 * (bp.x + s * bn.x), 0.5 * (bp.y - s * bn.y)};
      O o;
      if (!sg) { o.x = al.x - be.y; o.y = al.y + be.x; }
      else { o.x = al.x + be.y; o.y = be.x - al.y; }
      X[((int64_t)am * g.L + (l - am)) * nc + sg * g.B + j0 + jj] = o;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void real_slots_to_coef_kernel(Geo g, int Breal, const double2* __restrict__ Y,
                                                                 double2* __restrict__ flm) {
  __shared__ double2 ty[2][8][65];  // [sign][complex map in chunk][order in chunk]
  const int l = blockIdx.y, am0 = 64 * (int)blockIdx.x;
  if (am0 > l) return;
  const int nam = min(64, l - am0 + 1);
  const int nc = g.ncols >> 1;
  const int64_t LL = (int64_t)g.L * g.L;
  for (int j0 = 0; j0 < g.B; j0 += 8) {
    const int nj = min(8, g.B - j0);
    for (int e = threadIdx.x; e < nam * 2 * nj; e += blockDim.x) {
      const int col = e % (2 * nj), ai = e / (2 * nj);
      const int sg = col / nj, jj = col - sg * nj;
      const int am = am0 + ai;
      const int c = (am == 0) ? jj : sg * g.B + jj;  // order 0: N is P
      ty[sg][jj][ai] = Y[((int64_t)am * g.L + (l - am)) * nc + j0 + c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * 2 * nj * nam; e += blockDim.x) {
      const int ai = e % nam, rest = e / nam;
      const int rr = rest % (2 * nj), sg = rest / (2 * nj);
      const int r = 2 * j0 + rr, am = am0 + ai;
      if (r >= Breal || (am == 0 && sg)) continue;
      const int jj = rr >> 1;
      const double2 P = ty[0][jj][ai], N = ty[1][jj][ai];
      const double s = sg ? ((am & 1) ? -1.0 : 1.0) : 1.0;
      // sg = 0: (P + conj N)/2 and (P - conj N)/(2i); sg = 1: the same with P, N swapped, times (-1)^m
      const double2 u = sg ? N : P, w = sg ? P : N;
      double2 v;
      if (rr & 1) { v.x = 0.5 * s * (u.y + w.y); v.y = -0.5 * s * (u.x - w.x); }
      else { v.x = 0.5 * s * (u.x + w.x); v.y = 0.5 * s * (u.y - w.y); }
      flm[(int64_t)r * LL + (int64_t)l * l + l + (sg ? -am : am)] = v;
    }
    __syncthreads();
  }
}

}  // namespace

// Workgroups of the coefficient transposes: the chunks of 64 orders of every degree.
int64_t transpose_blocks(int L) {
  int64_t n = 0;
  for (int l = 0; l < L; ++l) n += l / 32 + 1;
  return n;
}

void launch_fwd_scatter(const Plan& p, const double* Y, double* flm, int64_t B, hipStream_t st, int64_t real_maps) {
  const Geo g = geo(p, B);
  if (real_maps > 0) {
    hipLaunchKernelGGL(real_slots_to_coef_kernel, dim3((unsigned)ceil_div(p.L, 64), p.L), dim3(256), 0, st, g,
                       (int)real_maps, reinterpret_cast<const double2*>(Y), reinterpret_cast<double2*>(flm));
    OSHT_HIP(hipGetLastError());
    return;
  }
  hipLaunchKernelGGL(coef_transpose_kernel<false>, dim3((unsigned)transpose_blocks(p.L)), dim3(256), 0, st, g,
                     reinterpret_cast<const double2*>(Y), reinterpret_cast<double2*>(flm));
  OSHT_HIP(hipGetLastError());
}

void launch_coef_to_slots(const Plan& p, const double* flm, double* X, int64_t B, hipStream_t st, bool f32,
                          int64_t real_maps = 0) {
  const Geo g = geo(p, B);
  if (real_maps > 0) {
    const dim3 rgrid((unsigned)ceil_div(p.L, 64), p.L);
    if (f32)
      hipLaunchKernelGGL(real_coef_to_slots_kernel<float2>, rgrid, dim3(256), 0, st, g, (int)real_maps,
                         reinterpret_cast<const double2*>(flm), reinterpret_cast<float2*>(X));
    else
      hipLaunchKernelGGL(real_coef_to_slots_kernel<double2>, rgrid, dim3(256), 0, st, g, (int)real_maps,
                         reinterpret_cast<const double2*>(flm), reinterpret_cast<double2*>(X));
    OSHT_HIP(hipGetLastError());
    return;
  }
  const dim3 grid((unsigned)transpose_blocks(p.L));
  if (f32)
    hipLaunchKernelGGL((coef_transpose_kernel<true, float2>), grid, dim3(256), 0, st, g,
                       reinterpret_cast<const double2*>(flm), reinterpret_cast<float2*>(X));
  else
    hipLaunchKernelGGL((coef_transpose_kernel<true, double2>), grid, dim3(256), 0, st, g,
                       reinterpret_cast<const double2*>(flm), reinterpret_cast<double2*>(X));
  OSHT_HIP(hipGetLastError());
}

void gemm_tasks_launch(Plan& p, const GemmTask* d_tasks, int count, GemmRole role, const char* prof_name,
                       hipStream_t st) {
  if (count <= 0) return;
  const int var = role == GemmRole::ApplyForward                                       ? p.gvar_fwd
                  : (role == GemmRole::ApplyInverse || role == GemmRole::ApplyInverse32) ? p.gvar_inv
                                                                                         : 0;
  if (p.prof.wants(prof_name)) {
    hipEvent_t e0 = p.prof.get(), e1 = p.prof.get();
    launch_gemm(role, p.tab->d_gdesc.as<GemmDesc>(), d_tasks, count, st, e0, e1, var);
    p.prof.stat(prof_name).pending.emplace_back(e0, e1);
    return;
  }
  launch_gemm(role, p.tab->d_gdesc.as<GemmDesc>(), d_tasks, count, st, nullptr, nullptr, var);
}

namespace {

// task range [first, count) of the GEMMs for direction dir, slots [s0, s1)
void task_range(const Plan& p, int dir, int s0, int s1, int& first, int& count) {
  const int d0 = dir * p.nslots + s0, d1 = dir * p.nslots + s1;
  int lo = 0, hi = (int)p.tab->h_gtask.size();
  {
    int a = 0, b = hi;
    while (a < b) { int mid = (a + b) / 2; if (p.tab->h_gtask[mid].desc < d0) a = mid + 1; else b = mid; }
    lo = a;
  }
  {
    int a = lo, b = hi;
    while (a < b) { int mid = (a + b) / 2; if (p.tab->h_gtask[mid].desc < d1) a = mid + 1; else b = mid; }
    hi = a;
  }
  first = lo;
  count = hi - lo;
}

void gemm_slots(Plan& p, int dir, int s0, int s1, hipStream_t st) {
  int first, count;
  task_range(p, dir, s0, s1, first, count);
  // inverse / forward read A or Q column-major; the adjoints read them transposed
  const GemmRole role = dir == kInv                        ? (p.fp32 ? GemmRole::ApplyInverse32 : GemmRole::ApplyInverse)
                        : (dir == kFwd || dir == kFwdAlias)  ? GemmRole::ApplyForward
                        : (dir == kCorr || dir == kCorrAlias) ? GemmRole::Correction
                                                              : GemmRole::Adjoint;
  gemm_tasks_launch(p, p.tab->d_gtask.as<GemmTask>() + first, count, role, kApplyName[dir], st);
}

// slots of level am: spin 0 -> [am, am+1); spin s -> {-am, +am}
void level_slots(const Plan& p, int am, int& s0, int& s1) {
  if (p.spin == 0) { s0 = am; s1 = am + 1; return; }
  const int c = p.L - 1;
  if (am == 0) { s0 = c; s1 = c + 1; return; }
  s0 = c - am; s1 = c + am + 1;  // contains the two slots at the ends only
}

}  // namespace

void run_inverse(Plan& p, const double* flm, double* f, int64_t B, hipStream_t st, int64_t real_maps) {
  ensure_workspace(p, B);
  const Geo g = geo(p, B);
  (void)g;
  {
    ProfScope ps(p.prof, "coef_to_slots", st);
    launch_coef_to_slots(p, flm, p.w_X.as<double>(), B, st, p.fp32, real_maps);
  }
  if (p.oz) {
    {
      ProfScope ps(p.prof, "split_digits", st);
      launch_oz_split_x(p, p.w_X.as<double>(), B, p.w_X8.as<int8_t>(), p.w_Xexp.as<int32_t>(), st);
    }
    const int n = (int)p.tab->h_oztask.size();
    const OzDesc* dd = p.tab->d_ozdesc.as<OzDesc>();
    const GemmTask* dt = p.tab->d_oztask.as<GemmTask>();
    if (p.prof.wants(kApplyName[kInv])) {
      hipEvent_t e0 = p.prof.get(), e1 = p.prof.get();
      launch_oz_apply(p, dd, dt, n, st, e0, e1);
      p.prof.stat(kApplyName[kInv]).pending.emplace_back(e0, e1);
    } else {
      launch_oz_apply(p, dd, dt, n, st);
    }
  } else {
    gemm_slots(p, kInv, 0, p.nslots, st);
  }
  {
    ProfScope ps(p.prof, "fold", st);
    launch_fold(p, p.w_Y.as<double>(), p.w_H.as<double>(), B, st);
  }
  ProfScope ps(p.prof, "ring_synthesis", st);
  launch_ring_synthesis(p, p.w_H.as<double>(), 0, f, B, st, real_maps);
}

void run_forward_levels(Plan& p, const double* f, double* flm, int64_t B, hipStream_t st, int64_t real_maps) {
  ensure_workspace(p, B);
  const Geo g = geo(p, B);
  {
    ProfScope ps(p.prof, "ring_analysis", st);
    launch_ring_analysis(p, f, p.w_H.as<double>(), B, true, st, real_maps);
  }
  const dim3 blk(256);
  for (int am = p.L - 1; am >= 0; --am) {
    int s0, s1;
    level_slots(p, am, s0, s1);
    const int R = p.L - am;
    const unsigned gx = (unsigned)ceil_div((int64_t)R * g.ncols, 256);
    if (p.spin == 0 || am == 0) {
      hipLaunchKernelGGL(fwd_gather_kernel, dim3(gx, s1 - s0), blk, 0, st, g, p.d_slots.as<Slot>(), s0,
                         p.w_H.as<double>(), p.w_Y.as<double>(), p.w_X.as<double>());
      OSHT_HIP(hipGetLastError());
      gemm_slots(p, kFwd, s0, s1, st);
      gemm_slots(p, kFwdAlias, s0, s1, st);
    } else {
      for (int sl : {s0, s1 - 1}) {
        hipLaunchKernelGGL(fwd_gather_kernel, dim3(gx, 1), blk, 0, st, g, p.d_slots.as<Slot>(), sl,
                           p.w_H.as<double>(), p.w_Y.as<double>(), p.w_X.as<double>());
        OSHT_HIP(hipGetLastError());
        gemm_slots(p, kFwd, sl, sl + 1, st);
        gemm_slots(p, kFwdAlias, sl, sl + 1, st);
      }
    }
  }
  launch_fwd_scatter(p, p.w_Y.as<double>(), flm, B, st, real_maps);
}

void run_inverse_adjoint(Plan& p, const double* fbar, double* flmbar, int64_t B, hipStream_t st) {
  ensure_workspace(p, B);
  const Geo g = geo(p, B);
  launch_ring_analysis(p, fbar, p.w_H.as<double>(), B, false, st);
  const dim3 grid((unsigned)ceil_div((int64_t)p.L * g.ncols, 256), (unsigned)p.nslots);
  hipLaunchKernelGGL(iadj_gather_kernel, grid, dim3(256), 0, st, g, p.d_slots.as<Slot>(), 0, p.w_H.as<double>(),
                     p.w_X.as<double>());
  OSHT_HIP(hipGetLastError());
  gemm_slots(p, kIadj, 0, p.nslots, st);
  launch_fwd_scatter(p, p.w_Y.as<double>(), flmbar, B, st, 0);
}

void run_forward_adjoint(Plan& p, const double* flmbar, double* fbar, int64_t B, hipStream_t st) {
  if (p.fb.b > 1) {
    run_forward_adjoint_blocked(p, flmbar, fbar, B, st);
    return;
  }
  ensure_workspace(p, B);
  const Geo g = geo(p, B);
  const dim3 blk(256);
  for (int am = 0; am < p.L; ++am) {
    int s0, s1;
    level_slots(p, am, s0, s1);
    const int rows = p.L;  // K + |m| <= L and R <= L
    const unsigned gx = (unsigned)ceil_div((int64_t)rows * g.ncols, 256);
    std::vector<int> list;
    if (p.spin == 0 || am == 0) list = {s0}; else list = {s0, s1 - 1};
    for (int sl : list) {
      hipLaunchKernelGGL(fadj_gather_kernel, dim3(gx, 1), blk, 0, st, g, p.d_slots.as<Slot>(), sl, flmbar,
                         p.w_H.as<double>(), p.w_X.as<double>());
      OSHT_HIP(hipGetLastError());
      gemm_slots(p, kFadj, sl, sl + 1, st);
      hipLaunchKernelGGL(fadj_scatter_kernel, dim3(gx, 1), blk, 0, st, g, p.d_slots.as<Slot>(), sl,
                         p.w_Y.as<double>(), p.w_H.as<double>());
      OSHT_HIP(hipGetLastError());
    }
  }
  launch_ring_synthesis(p, p.w_H.as<double>(), 1, fbar, B, st);
}

void run_forward(Plan& p, const double* f, double* flm, int64_t B, hipStream_t st, int64_t real_maps) {
  if (p.fb.b > 1) run_forward_blocked(p, f, flm, B, st, real_maps);
  else run_forward_levels(p, f, flm, B, st, real_maps);
}

// ---------------------------------------------------------------- real maps
// Spin-0 maps with real samples have coefficients with the symmetry
// f_{l,-m} = (-1)^m conj(f_{l,m}), from the harmonics' conjugation rule
// (Eq. yellm:conj, appendix on spherical harmonics).  Two real maps a and b are transformed as the one complex map
// z = a + i b: the inverse of z has real part a and imaginary part b, and
// the forward of z gives a_lm = (z_lm + R(z)_lm)/2 and
// b_lm = (z_lm - R(z)_lm)/(2i) with R(z)_lm = (-1)^m conj(z_{l,-m}).  Half
// the right-hand-side columns, ring DFTs and matrix work per real map.

namespace {

void check_real(const Plan& p) {
  OSHT_CHECK(p.spin == 0, OSHT_ENOTSUP, "real-map transforms are defined for spin 0 only");
}

}  // namespace

// Two real maps per complex transform: the ring DFTs read and write the real
// samples directly, and the coefficient transposes pack and unpack the
// conjugation-symmetric parts (no extra passes).
void run_forward_real(Plan& p, const double* f, double* flm, int64_t B, hipStream_t st) {
  check_real(p);
  run_forward(p, f, flm, (B + 1) / 2, st, B);
}

void run_inverse_real(Plan& p, const double* flm, double* f, int64_t B, hipStream_t st) {
  check_real(p);
  run_inverse(p, flm, f, (B + 1) / 2, st, B);
}

// ---------------------------------------------------------------- checks
namespace {

// Any NaN / Inf among x[0, n) sets *flag (plain store: every writer writes 1).
__global__ __launch_bounds__(256) void finite_scan_kernel(const double* __restrict__ x, int64_t n,
                                                          int32_t* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (__ballot(bad) && (threadIdx.x & 63) == 0) *flag = 1;
}

// splitmix64 (Steele, Lea & Flood, OOPSLA 2014): a fixed pseudo-random
// stream for the self-check's input.
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

}  // namespace

void launch_finite_scan(Plan& p, const double* x, int64_t n, hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<int64_t>(std::max<int64_t>(ceil_div(n, 256 * 8), 1), 4096);
  hipLaunchKernelGGL(finite_scan_kernel, dim3(blocks), dim3(256), 0, st, x, n, p.d_status.as<int32_t>());
  OSHT_HIP(hipGetLastError());
}

// The forward is exact on band-limited samples, so forward(inverse(a)) - a
// measures the rounding that the order-by-order chain of Procedure 1
// amplifies on this plan.  Run in FP64 on one map with entries uniform in
// [-1, 1) + i[-1, 1) (zero for l < |s|); synchronous, on the null stream.
void forward_self_check(Plan& p) {
  const int64_t n = (int64_t)p.L * p.L;
  std::vector<double> a(2 * n), back(2 * n);
  uint64_t seed = 0x5eed0000ull + (uint64_t)p.L * 131u + (uint64_t)(p.spin + 64);
  const int as = std::abs(p.spin);
  int l = 0;
  for (int64_t i = 0; i < n; ++i) {
    if ((int64_t)(l + 1) * (l + 1) <= i) ++l;  // i = l^2 + l + m
    for (int part = 0; part < 2; ++part) {
      const double u = (double)(splitmix64(seed) >> 11) * 0x1.0p-53;  // [0, 1)
      a[2 * i + part] = l < as ? 0.0 : 2.0 * u - 1.0;
    }
  }
  DevBuf d_a, d_f, d_g;
  d_a.alloc(sizeof(double) * 2 * n);
  d_f.alloc(sizeof(double) * 2 * n);
  d_g.alloc(sizeof(double) * 2 * n);
  OSHT_HIP(hipMemcpy(d_a.p, a.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice));
  run_inverse(p, d_a.as<double>(), d_f.as<double>(), 1, 0);
  run_forward(p, d_f.as<double>(), d_g.as<double>(), 1, 0);
  OSHT_HIP(hipMemcpy(back.data(), d_g.p, sizeof(double) * 2 * n, hipMemcpyDeviceToHost));
  double num = 0.0, den = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double dr = back[2 * i] - a[2 * i], di = back[2 * i + 1] - a[2 * i + 1];
    const double d = std::sqrt(dr * dr + di * di);
    num = (d == d && num == num) ? std::max(num, d) : NAN;
    den = std::max(den, std::sqrt(a[2 * i] * a[2 * i] + a[2 * i + 1] * a[2 * i + 1]));
  }
  p.fwd_check_err = den > 0.0 ? num / den : num;
  p.fwd_unstable = p.spin != 0 && !(p.fwd_check_err <= kSpinForwardStableErr && p.max_resid <= kMaxInvResidual);
}

}  // namespace osht
