// Plan construction on the GPU: Legendre / Wigner blocks (Sec. III-F/G),
// per-order inversion of P_m by Newton-Schulz iteration, and the stacked
// forward operators Q_m = [P_m^{-1}; A_m^top P_m^{-1}].
//
// Block A_m (slot layout, column-major, rows = rings k = 0..L-1, columns =
// degrees l = l0..L-1):  A_m[k, i] = sY_{l0+i}^m(theta_k, 0).
// P_m = rows k >= |m| of A_m (Eq. Y_matrix without the common 2 pi), the
// "top" rows k < |m| evaluate order m on the rings where it aliases
// (Eq. signal_subset).  Forward operator per slot:
//     Q_m = [ X_m ; A_m^top X_m ],  X_m = P_m^{-1} (P_m^+ when |m| < |s|)
// so that one product Q_m g_m yields the order-m coefficients and the
// values G'_m(theta_k) on the rings k < |m| that later orders subtract.

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "common.hpp"
#include "host_util.hpp"

namespace osht {

namespace {

constexpr double kBig = 0x1p256, kSmall = 0x1p-256;

// ---------------------------------------------------------------- Legendre
// Spin 0, slot am, ring k: upward recurrence in l from the seed
// Pt[am, am] = prod_{i=1..am} (-sqrt((2i+1)/(2i)) sin theta) / sqrt(4 pi),
// with values carried as mantissa * 2^e while below the double range.
__global__ __launch_bounds__(256) void legendre_s0_kernel(int L, const double* __restrict__ cs,
                                                          const double* __restrict__ sn, const Slot* __restrict__ slots,
                                                          double* __restrict__ A) {
  const int am = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  const Slot sl = slots[am];
  double* out = A + sl.offA + k;
  const double x = cs[k], y = sn[k];
  double p = 0.28209479177387814347;  // 1/sqrt(4 pi)
  int e = 0;
  for (int i = 1; i <= am && p != 0.0; ++i) {
    p *= -sqrt((2.0 * i + 1.0) / (2.0 * i)) * y;
    if (fabs(p) < kSmall && p != 0.0) {
      int de;
      p = frexp(p, &de);
      e += de;
    }
  }
  double prev = 0.0, cur = p;
  out[0] = ldexp(cur, e);
  for (int l = am; l < L - 1; ++l) {
    const double den = (double)(l + 1) * (l + 1) - (double)am * am;
    const double a = sqrt((2.0 * l + 1.0) * (2.0 * l + 3.0) / den);
    const double b = (l == am) ? 0.0 : sqrt((2.0 * l + 3.0) * ((double)l * l - (double)am * am) / ((2.0 * l - 1.0) * den));
    const double nxt = a * x * cur - b * prev;
    prev = cur;
    cur = nxt;
    const double mag = fmax(fabs(prev), fabs(cur));
    if (mag > kBig) { prev *= kSmall; cur *= kSmall; e += 256; }
    else if (mag < kSmall && mag > 0.0) { prev *= kBig; cur *= kBig; e -= 256; }
    out[(int64_t)(l + 1 - am) * sl.ldA] = ldexp(cur, e);
  }
}

// Spin s, slot for signed order m, ring k:
// sY_l^m(theta, 0) = (-1)^s sqrt((2l+1)/(4 pi)) d^l_{m,-s}(theta), with the
// Wigner-d recurrence in l for fixed (a, b) = (m, -s) started at
// j = max(|a|, |b|) from the single surviving term of Wigner's sum:
//   d^j_{ab} = sign * sqrt(C(2j, j+c)) cos^p(theta/2) sin^q(theta/2).
__global__ __launch_bounds__(256) void legendre_spin_kernel(int L, int s, const double* __restrict__ cs,
                                                            const double* __restrict__ ch, const double* __restrict__ sh,
                                                            const Slot* __restrict__ slots, double* __restrict__ A) {
  const int slot = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  const Slot sl = slots[slot];
  const int a = sl.m, b = -s;
  const int j0 = sl.l0;
  double* out = A + sl.offA + k;
  int sign, pc, ps, c;
  if (abs(a) >= abs(b)) {
    c = b;
    if (a == j0) { sign = ((j0 - b) & 1) ? -1 : 1; pc = j0 + b; ps = j0 - b; }
    else { sign = 1; pc = j0 - b; ps = j0 + b; }
  } else {
    c = a;
    if (b == j0) { sign = 1; pc = j0 + a; ps = j0 - a; }
    else { sign = ((j0 + a) & 1) ? -1 : 1; pc = j0 - a; ps = j0 + a; }
  }
  // C(2j, j+c) = prod_{i=1}^{j-c} (j+c+i)/i, taken under a square root
  double p = (double)sign;
  int e = 0;
  auto renorm = [&]() {
    if (p != 0.0 && (fabs(p) < kSmall || fabs(p) > kBig)) {
      int de;
      p = frexp(p, &de);
      e += de;
    }
  };
  for (int i = 1; i <= j0 - c; ++i) { p *= sqrt((double)(j0 + c + i) / (double)i); renorm(); }
  const double cv = ch[k], sv = sh[k];
  for (int i = 0; i < pc && p != 0.0; ++i) { p *= cv; renorm(); }
  for (int i = 0; i < ps && p != 0.0; ++i) { p *= sv; renorm(); }
  const double sgn_s = (s & 1) ? -1.0 : 1.0;
  const double inv4pi = 0.07957747154594766788;  // 1/(4 pi)
  double prev = 0.0, cur = p;
  out[0] = sgn_s * sqrt((2.0 * j0 + 1.0) * inv4pi) * ldexp(cur, e);
  const double x = cs[k];
  for (int j = j0; j < L - 1; ++j) {
    double nxt;
    if (j == 0) {
      nxt = x * cur;
    } else {
      const double dn = (double)j * sqrt(((double)(j + 1) * (j + 1) - (double)a * a) * ((double)(j + 1) * (j + 1) - (double)b * b));
      const double c1 = (2.0 * j + 1.0) * ((double)j * (j + 1) * x - (double)a * b);
      const double c2 = (double)(j + 1) * sqrt(((double)j * j - (double)a * a) * ((double)j * j - (double)b * b));
      nxt = (c1 * cur - c2 * prev) / dn;
    }
    prev = cur;
    cur = nxt;
    const double mag = fmax(fabs(prev), fabs(cur));
    if (mag > kBig) { prev *= kSmall; cur *= kSmall; e += 256; }
    else if (mag < kSmall && mag > 0.0) { prev *= kBig; cur *= kBig; e -= 256; }
    const int l = j + 1;
    out[(int64_t)(l - j0) * sl.ldA] = sgn_s * sqrt((2.0 * l + 1.0) * inv4pi) * ldexp(cur, e);
  }
}

// ---------------------------------------------------------------- Newton-Schulz
// Per slot: ||P||_1 ||P||_inf, P = rows |m|.. of A (R x K).
__global__ __launch_bounds__(256) void pnorms_kernel(const Slot* __restrict__ slots, int slot0, const double* __restrict__ A,
                                                     double* __restrict__ out) {
  const Slot sl = slots[slot0 + blockIdx.x];
  const int am = sl.m < 0 ? -sl.m : sl.m;
  const double* P = A + sl.offA + am;
  __shared__ double red[2][256];
  double cmax = 0.0, rmax = 0.0;
  for (int j = threadIdx.x; j < sl.K; j += blockDim.x) {  // column sums
    double acc = 0.0;
    for (int i = 0; i < sl.R; ++i) acc += fabs(P[(int64_t)j * sl.ldA + i]);
    cmax = fmax(cmax, acc);
  }
  for (int i = threadIdx.x; i < sl.R; i += blockDim.x) {  // row sums
    double acc = 0.0;
    for (int j = 0; j < sl.K; ++j) acc += fabs(P[(int64_t)j * sl.ldA + i]);
    rmax = fmax(rmax, acc);
  }
  red[0][threadIdx.x] = cmax;
  red[1][threadIdx.x] = rmax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = red[0][0];
    out[2 * blockIdx.x + 1] = red[1][0];
  }
}

// X0 = alpha P^T into the top K rows of Q (K x R, column-major, ld ldQ).
__global__ __launch_bounds__(256) void ns_init_kernel(const Slot* __restrict__ slots, int slot0, const double* __restrict__ A,
                                                      double* __restrict__ Q, const double* __restrict__ norms) {
  const Slot sl = slots[slot0 + blockIdx.y];
  const int am = sl.m < 0 ? -sl.m : sl.m;
  const double alpha = 1.0 / (norms[2 * blockIdx.y] * norms[2 * blockIdx.y + 1]);
  const int64_t total = (int64_t)sl.K * sl.R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % sl.K), j = (int)(e / sl.K);  // X[i][j] = alpha P[j][i]
    Q[sl.offQ + (int64_t)j * sl.ldQ + i] = alpha * A[sl.offA + (int64_t)i * sl.ldA + am + j];
  }
}

// Y = scale * X for a K x R block per slot: X at Q top (ld ldQ) or at a
// packed scratch block (ld K); direction chosen by `to_q`.
__global__ __launch_bounds__(256) void ns_copy_kernel(const Slot* __restrict__ slots, int slot0, double* __restrict__ Q,
                                                      double* __restrict__ scr, const int64_t* __restrict__ offXn,
                                                      double scale, int to_q) {
  const Slot sl = slots[slot0 + blockIdx.y];
  const int64_t total = (int64_t)sl.K * sl.R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % sl.K), j = (int)(e / sl.K);
    double* q = Q + sl.offQ + (int64_t)j * sl.ldQ + i;
    double* x = scr + offXn[blockIdx.y] + e;
    if (to_q) *q = scale * (*x); else *x = scale * (*q);
  }
}

// As ns_copy_kernel (scale 1) for the slots whose flag is set: keeps the
// best iterate of each slot in scratch (to_q = 0) or restores it (to_q = 1).
__global__ __launch_bounds__(256) void ns_keep_kernel(const Slot* __restrict__ slots, int slot0, double* __restrict__ Q,
                                                      double* __restrict__ scr, const int64_t* __restrict__ offXb,
                                                      const int32_t* __restrict__ flag, int to_q) {
  if (!flag[blockIdx.y]) return;  // uniform over the workgroup
  const Slot sl = slots[slot0 + blockIdx.y];
  const int64_t total = (int64_t)sl.K * sl.R;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % sl.K), j = (int)(e / sl.K);
    double* q = Q + sl.offQ + (int64_t)j * sl.ldQ + i;
    double* x = scr + offXb[blockIdx.y] + e;
    if (to_q) *q = *x; else *x = *q;
  }
}

// max_ij |E_ij - delta_ij| for E = X P (K x K packed, ld K) per slot.
__global__ __launch_bounds__(256) void ns_resid_kernel(const Slot* __restrict__ slots, int slot0, const double* __restrict__ scr,
                                                       const int64_t* __restrict__ offE, double* __restrict__ out) {
  const Slot sl = slots[slot0 + blockIdx.x];
  const double* E = scr + offE[blockIdx.x];
  const int64_t total = (int64_t)sl.K * sl.K;
  double mx = 0.0;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int i = (int)(e % sl.K), j = (int)(e / sl.K);
    const double v = E[e] - (i == j ? 1.0 : 0.0);
    mx = fmax(mx, (v != v) ? INFINITY : fabs(v));
  }
  __shared__ double red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// ||X||_1 (max column abs sum of the K x R block at Q top) per slot.
__global__ __launch_bounds__(256) void xnorm1_kernel(const Slot* __restrict__ slots, int slot0, const double* __restrict__ Q,
                                                     double* __restrict__ out) {
  const Slot sl = slots[slot0 + blockIdx.x];
  double mx = 0.0;
  for (int j = threadIdx.x; j < sl.R; j += blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < sl.K; ++i) acc += fabs(Q[sl.offQ + (int64_t)j * sl.ldQ + i]);
    mx = fmax(mx, acc);
  }
  __shared__ double red[256];
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

template <class T>
void put(DevBuf& d, const std::vector<T>& h) {
  d.reserve(h.size() * sizeof(T));
  if (!h.empty()) OSHT_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

// Newton-Schulz for the slots [s0, s1): X <- 2X - X (P X), started from
// X0 = P^T / (||P||_1 ||P||_inf); stops when max |X P - I| no longer
// improves.  Each slot keeps the iterate with its smallest residual (copied
// aside whenever the residual falls), and that iterate is what ends in the
// top K rows of Q_m; returns the largest of those per-slot residuals and the
// 1-norm condition estimates via kappa_out.
double newton_schulz(Plan& p, int s0, int s1, DevBuf& scratch, std::vector<double>& kappa_out) {
  const int ns = s1 - s0;
  const Slot* d_slots = p.d_slots.as<Slot>();
  double* A = p.d_A.as<double>();
  double* Q = p.d_Q.as<double>();
  std::vector<int64_t> offT(ns), offXn(ns), offE(ns), offXb(ns);
  int64_t tot = 0;
  for (int i = 0; i < ns; ++i) {
    const Slot& sl = p.slots[s0 + i];
    offT[i] = tot; tot += (int64_t)sl.R * sl.R;
    offXn[i] = tot; tot += (int64_t)sl.K * sl.R;
    offE[i] = tot; tot += (int64_t)sl.K * sl.K;
    offXb[i] = tot; tot += (int64_t)sl.K * sl.R;
  }
  scratch.reserve(tot * sizeof(double));
  double* scr = scratch.as<double>();
  DevBuf d_offXn, d_offE, d_offXb, d_flag, d_norms, d_out;
  upload(d_offXn, offXn);
  upload(d_offE, offE);
  upload(d_offXb, offXb);
  d_flag.alloc(sizeof(int32_t) * ns);
  d_norms.alloc(sizeof(double) * 2 * ns);
  d_out.alloc(sizeof(double) * ns);
  std::vector<GemmDesc> dPX(ns), dXT(ns), dXP(ns);
  for (int i = 0; i < ns; ++i) {
    const Slot& sl = p.slots[s0 + i];
    const int am = std::abs(sl.m);
    const double* P = A + sl.offA + am;
    double* X = Q + sl.offQ;
    double* T = scr + offT[i];
    double* Xn = scr + offXn[i];
    double* E = scr + offE[i];
    dPX[i] = GemmDesc{P, X, T, 1, sl.ldA, 1, sl.ldQ, 1, sl.R, sl.R, sl.R, sl.K, 0, 1.0, 0.0};
    dXT[i] = GemmDesc{X, T, Xn, 1, sl.ldQ, 1, sl.R, 1, sl.K, sl.K, sl.R, sl.R, 0, -1.0, 1.0};
    dXP[i] = GemmDesc{X, P, E, 1, sl.ldQ, 1, sl.ldA, 1, sl.K, sl.K, sl.K, sl.R, 0, 1.0, 0.0};
  }
  std::vector<GemmTask> tPX, tXT, tXP;
  gemm_tasks(dPX, tPX);
  gemm_tasks(dXT, tXT);
  gemm_tasks(dXP, tXP);
  DevBuf gPX, gXT, gXP, kPX, kXT, kXP;
  upload(gPX, dPX); upload(gXT, dXT); upload(gXP, dXP);
  upload(kPX, tPX); upload(kXT, tXT); upload(kXP, tXP);
  hipLaunchKernelGGL(pnorms_kernel, dim3(ns), dim3(256), 0, 0, d_slots, s0, A, d_norms.as<double>());
  OSHT_HIP(hipGetLastError());
  std::vector<double> norms(2 * ns);
  OSHT_HIP(hipMemcpy(norms.data(), d_norms.p, sizeof(double) * 2 * ns, hipMemcpyDeviceToHost));
  hipLaunchKernelGGL(ns_init_kernel, dim3(64, ns), dim3(256), 0, 0, d_slots, s0, A, Q, d_norms.as<double>());
  OSHT_HIP(hipGetLastError());
  std::vector<double> res(ns), best_slot(ns, INFINITY);
  std::vector<int32_t> keep(ns);
  double last = INFINITY;
  int stall = 0;
  for (int it = 0; it < 120; ++it) {
    launch_gemm(GemmRole::Plan, gPX.as<GemmDesc>(), kPX.as<GemmTask>(), (int)tPX.size(), 0);
    hipLaunchKernelGGL(ns_copy_kernel, dim3(64, ns), dim3(256), 0, 0, d_slots, s0, Q, scr, d_offXn.as<int64_t>(), 2.0, 0);
    launch_gemm(GemmRole::Plan, gXT.as<GemmDesc>(), kXT.as<GemmTask>(), (int)tXT.size(), 0);
    hipLaunchKernelGGL(ns_copy_kernel, dim3(64, ns), dim3(256), 0, 0, d_slots, s0, Q, scr, d_offXn.as<int64_t>(), 1.0, 1);
    OSHT_HIP(hipGetLastError());
    if (it < 8) continue;
    launch_gemm(GemmRole::Plan, gXP.as<GemmDesc>(), kXP.as<GemmTask>(), (int)tXP.size(), 0);
    hipLaunchKernelGGL(ns_resid_kernel, dim3(ns), dim3(256), 0, 0, d_slots, s0, scr, d_offE.as<int64_t>(), d_out.as<double>());
    OSHT_HIP(hipGetLastError());
    OSHT_HIP(hipMemcpy(res.data(), d_out.p, sizeof(double) * ns, hipMemcpyDeviceToHost));
    double mx = 0.0;
    bool any = false;
    for (int i = 0; i < ns; ++i) {
      const double r = res[i] == res[i] ? res[i] : INFINITY;
      mx = std::max(mx, r);
      keep[i] = r < best_slot[i] ? 1 : 0;
      if (keep[i]) { best_slot[i] = r; any = true; }
    }
    if (any) {
      OSHT_HIP(hipMemcpy(d_flag.p, keep.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice));
      hipLaunchKernelGGL(ns_keep_kernel, dim3(64, ns), dim3(256), 0, 0, d_slots, s0, Q, scr, d_offXb.as<int64_t>(),
                         d_flag.as<int32_t>(), 0);
      OSHT_HIP(hipGetLastError());
    }
    if (mx < 1e-15) break;
    // The max-entry residual of a large P_m can sit near 1/n for many
    // iterations before the quadratic phase (the smallest singular value is
    // spread over n entries), so only a residual already at rounding level
    // that stops halving ends the iteration.
    if (mx < 1e-10 && mx > 0.5 * last) { if (++stall >= 2) break; } else stall = 0;
    last = mx;
  }
  // restore each slot's best iterate (slots whose residual was never finite
  // keep the last one; the caller rejects them)
  double best = 0.0;
  for (int i = 0; i < ns; ++i) {
    keep[i] = best_slot[i] < INFINITY ? 1 : 0;
    best = std::max(best, best_slot[i]);
  }
  OSHT_HIP(hipMemcpy(d_flag.p, keep.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(ns_keep_kernel, dim3(64, ns), dim3(256), 0, 0, d_slots, s0, Q, scr, d_offXb.as<int64_t>(),
                     d_flag.as<int32_t>(), 1);
  OSHT_HIP(hipGetLastError());
  hipLaunchKernelGGL(xnorm1_kernel, dim3(ns), dim3(256), 0, 0, d_slots, s0, Q, d_out.as<double>());
  OSHT_HIP(hipGetLastError());
  std::vector<double> xn(ns);
  OSHT_HIP(hipMemcpy(xn.data(), d_out.p, sizeof(double) * ns, hipMemcpyDeviceToHost));
  for (int i = 0; i < ns; ++i) kappa_out.push_back(norms[2 * i] * xn[i]);
  return best;
}

// round-to-nearest FP32 copy
__global__ void narrow_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

}  // namespace

int64_t Plan::device_bytes() const {
  size_t n = 0;
  for (const DevBuf* b : {&d_cos, &d_sin, &d_cosh, &d_sinh, &d_slots, &d_A, &d_Q, &d_A32, &d_Q32, &d_rings, &d_chirp,
                          &d_twiddle, &d_chirp_tab, &w_X, &w_Y, &w_H, &w_T, &w_D, &d_status, &d_A8, &d_Aexp, &d_ozoff, &d_ozrow, &d_ozkstart, &d_ring_cut, &w_X8, &w_Xexp,
                          &fb.d_slot_list, &fb.d_lev_ptr, &fb.d_unk_slot, &fb.d_unk_r, &fb.d_unk_m, &fb.d_src_ptr,
                          &fb.d_src_slot, &fb.d_src_row, &fb.d_src_m, &fb.d_w_ptr, &fb.d_w_col, &fb.d_w_val,
                          &fb.d_wide_slot, &fb.d_wide_row, &fb.d_wt_ptr, &fb.d_wt_row, &fb.d_wt_val, &fb.d_minv,
                          &fb.d_src_yrow})
    n += b->bytes;
  for (const auto& t : tabs) n += t->bytes();
  return (int64_t)n;
}

// One workgroup per slot: the largest |A_m[k, l]| over the degrees of each
// ring k; orders whose row reaches 2^-80 raise ring k's cut to |m| + 1.  The
// values left out sum to below 2^-80 sum_l |x_l| per bin, far under FP64
// resolution of bins of that scale (Sec. III-F: on a ring near a pole
// P_l^m(theta) decays exponentially once |m| > l sin(theta)).
__global__ __launch_bounds__(256) void ring_cut_kernel(const Slot* __restrict__ slots, const double* __restrict__ A,
                                                       int L, int32_t* __restrict__ cut) {
  const Slot sl = slots[blockIdx.x];
  const int am = sl.m < 0 ? -sl.m : sl.m;
  const double* Ac = A + sl.offA;
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    double mx = 0.0;
    for (int l = 0; l < sl.K; ++l) mx = fmax(mx, fabs(Ac[k + (int64_t)l * sl.ldA]));
    if (mx >= 0x1p-80) atomicMax(&cut[k], am + 1);
  }
}

void build_ring_cut(Plan& p) {
  std::vector<int32_t> cut(p.L, 0);
  const char* e = std::getenv("OSHT_RING_CUT");
  if (e && std::atoi(e) == 0) {
    std::fill(cut.begin(), cut.end(), p.L);
  } else {
    upload(p.d_ring_cut, cut);
    hipLaunchKernelGGL(ring_cut_kernel, dim3((unsigned)p.nslots), dim3(256), 0, 0, p.d_slots.as<Slot>(),
                       p.d_A.as<double>(), p.L, p.d_ring_cut.as<int32_t>());
    OSHT_HIP(hipGetLastError());
    OSHT_HIP(hipMemcpy(cut.data(), p.d_ring_cut.p, sizeof(int32_t) * p.L, hipMemcpyDeviceToHost));
    for (int32_t& c : cut) c = std::max(c, 1);  // order 0 always stays
  }
  p.h_ring_cut = cut;
  upload(p.d_ring_cut, cut);
}

void build_plan(Plan& p) {
  const int L = p.L, s = p.spin;
  // ring trigonometry
  std::vector<double> cs(L), sn(L), chv(L), shv(L);
  for (int k = 0; k < L; ++k) ring_trig(L, p.numer[k], &cs[k], &sn[k], &chv[k], &shv[k]);
  upload(p.d_cos, cs);
  upload(p.d_sin, sn);
  upload(p.d_cosh, chv);
  upload(p.d_sinh, shv);
  // slots
  p.slots.clear();
  const int ldA = round_up(L, 8);
  int64_t offA = 0, offQ = 0;
  auto add_slot = [&](int m) {
    Slot sl{};
    sl.m = m;
    sl.l0 = std::max(std::abs(m), std::abs(s));
    sl.K = L - sl.l0;
    sl.R = L - std::abs(m);
    sl.ldA = ldA;
    sl.offA = offA;
    offA += (int64_t)ldA * sl.K;
    sl.ldQ = round_up(sl.K + std::abs(m), 8);
    sl.offQ = offQ;
    offQ += (int64_t)sl.ldQ * sl.R;
    p.slots.push_back(sl);
  };
  if (s == 0) {
    for (int am = 0; am < L; ++am) add_slot(am);
    p.ncols_per_map = 4;
  } else {
    for (int m = -(L - 1); m <= L - 1; ++m) add_slot(m);
    p.ncols_per_map = 2;
  }
  p.nslots = (int)p.slots.size();
  upload(p.d_slots, p.slots);
  p.d_A.alloc(sizeof(double) * offA);
  p.d_Q.alloc(sizeof(double) * offQ);
  OSHT_HIP(hipMemset(p.d_A.p, 0, p.d_A.bytes));
  OSHT_HIP(hipMemset(p.d_Q.p, 0, p.d_Q.bytes));
  // Legendre / Wigner blocks
  const dim3 grid((unsigned)ceil_div(L, 256), (unsigned)p.nslots);
  if (s == 0) {
    hipLaunchKernelGGL(legendre_s0_kernel, grid, dim3(256), 0, 0, L, p.d_cos.as<double>(), p.d_sin.as<double>(),
                       p.d_slots.as<Slot>(), p.d_A.as<double>());
  } else {
    hipLaunchKernelGGL(legendre_spin_kernel, grid, dim3(256), 0, 0, L, s, p.d_cos.as<double>(), p.d_cosh.as<double>(),
                       p.d_sinh.as<double>(), p.d_slots.as<Slot>(), p.d_A.as<double>());
  }
  OSHT_HIP(hipGetLastError());
  // the fold of every inverse from here on (the self-check's included) reads it
  build_ring_cut(p);
  // Newton-Schulz inverses, in chunks bounded by a scratch budget
  DevBuf scratch;
  const int64_t budget = (int64_t)1 << 28;  // doubles (2 GiB)
  std::vector<double> kap;
  p.max_resid = 0.0;
  for (int s0 = 0; s0 < p.nslots;) {
    int64_t need = 0;
    int s1 = s0;
    while (s1 < p.nslots) {
      const Slot& sl = p.slots[s1];
      const int64_t n1 = (int64_t)sl.R * sl.R + 2 * (int64_t)sl.K * sl.R + (int64_t)sl.K * sl.K;
      if (s1 > s0 && need + n1 > budget) break;
      need += n1;
      ++s1;
    }
    p.max_resid = std::max(p.max_resid, newton_schulz(p, s0, s1, scratch, kap));
    s0 = s1;
  }
  scratch.release();
  p.max_kappa = 0.0;
  for (double k : kap) p.max_kappa = std::max(p.max_kappa, k);
  // Spin 0: converged inverses of the greedy placement reach 1e-15 .. 3e-14
  // up to L = 2048; a residual above 1e-10 means some P_m is numerically
  // singular for FP64 (the alternating placement from L = 128 up stalls at
  // O(0.1)), and the plan is refused.  Spin != 0: the inverses feed only the
  // forward (the inverse and its adjoint read A_m), so a residual above the
  // bar marks the forward unusable instead (spin 2 at L = 2048 stalls near
  // 2e-5), together with the round-trip self-check below.
  if (p.spin == 0)
    OSHT_CHECK(p.max_resid <= kMaxInvResidual, OSHT_ESINGULAR,
               "per-order inversion did not converge (max |X P - I| = " + std::to_string(p.max_resid) + ")");
  // bottom rows of Q: A^top X
  std::vector<GemmDesc> dC;
  for (int i = 0; i < p.nslots; ++i) {
    const Slot& sl = p.slots[i];
    const int am = std::abs(sl.m);
    if (am == 0) continue;
    const double* At = p.d_A.as<double>() + sl.offA;
    const double* X = p.d_Q.as<double>() + sl.offQ;
    double* C = p.d_Q.as<double>() + sl.offQ + sl.K;
    dC.push_back(GemmDesc{At, X, C, 1, sl.ldA, 1, sl.ldQ, 1, sl.ldQ, am, sl.R, sl.K, 0, 1.0, 0.0});
  }
  if (!dC.empty()) {
    std::vector<GemmTask> tC;
    gemm_tasks(dC, tC);
    DevBuf gd, gt;
    upload(gd, dC);
    upload(gt, tC);
    launch_gemm(GemmRole::Plan, gd.as<GemmDesc>(), gt.as<GemmTask>(), (int)tC.size(), 0);
    OSHT_HIP(hipDeviceSynchronize());
  }
  build_chirps(p);
  // Block size of the forward sweep (or OSHT_FWD_BLOCK), shrunk until the
  // alias system fits the delta solve's LDS: 48 levels from L = 768 up, else
  // 32 (what the autotuner picks on MI355X at L = 1024 and 512).
  int b = p.L >= 768 ? 48 : 32;
  const char* env = std::getenv("OSHT_FWD_BLOCK");
  if (env) b = std::max(1, std::atoi(env));
  // OSHT_DELTA_DENSE=0: level-by-level substitution instead of the
  // precomputed (I + W)^{-1}
  if (const char* ed = std::getenv("OSHT_DELTA_DENSE")) p.fb.dense = std::atoi(ed) != 0;
  while (!fwd_blocks_fit(p, b) && b > 1) b = std::max(1, b * 3 / 4);
  // the forward self-check runs in FP64, before the FP32 copies replace A_m
  {
    const bool f32 = p.fp32, f32q = p.fp32_fwd;
    const int oz = p.oz;
    p.fp32 = p.fp32_fwd = false;
    p.oz = 0;
    forward_self_check(p);
    invalidate_tables(p);
    p.fp32 = f32;
    p.fp32_fwd = f32q;
    p.oz = oz;
  }
  if (p.oz) build_oz_planes(p);
  if (p.flags & OSHT_CHECK_FINITE) {
    p.d_status.alloc(sizeof(int32_t));
    OSHT_HIP(hipMemset(p.d_status.p, 0, sizeof(int32_t)));
  }
  // FP32 copies at the same element offsets.  FP32 plans release A_m; Q_m
  // stays in FP64 (the forward's alias rows A_m^top P_m^{-1} and the forward
  // adjoint always use it), with an FP32 copy for the coefficient rows when
  // the forward's coefficient tiles run in FP32
  auto narrow = [](DevBuf& src, DevBuf& dst, bool release) {
    const int64_t n = (int64_t)(src.bytes / sizeof(double));
    dst.alloc(sizeof(float) * std::max<int64_t>(n, 1));
    hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)std::min<int64_t>(std::max<int64_t>(ceil_div(n, 256), 1), 8192)),
                       dim3(256), 0, 0, src.as<double>(), dst.as<float>(), n);
    OSHT_HIP(hipGetLastError());
    OSHT_HIP(hipDeviceSynchronize());
    if (release) src.release();
  };
  if (p.fp32) narrow(p.d_A, p.d_A32, true);
  if (p.fp32_fwd) narrow(p.d_Q, p.d_Q32, false);
  if ((p.flags & OSHT_TUNE) && !env) autotune(p);
  // forced stream shapes of the forward and inverse applies, "fwd,inv" (tests)
  if (const char* ev = std::getenv("OSHT_GEMM_VAR")) {
    int f = 0, i = 0;
    if (std::sscanf(ev, "%d,%d", &f, &i) == 2 && f >= 0 && f < kGemmVars && i >= 0 && i < kGemmVars) {
      p.gvar_fwd = f;
      p.gvar_inv = i;
    }
  }
  OSHT_HIP(hipDeviceSynchronize());
}

}  // namespace osht
