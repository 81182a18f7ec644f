// Ring DFTs of the odd lengths n = 2k+1 (k = 0..L-1) by Bluestein's chirp-z
// algorithm on power-of-two FFTs held in registers.
//
// Analysis (ring k, one map):      H[q] = s * sum_j f_j e^{-2 pi i q j / n}
// Synthesis:                       f_j  =     sum_q H[q] e^{+2 pi i q j / n}
// With w_t = e^{-i pi t^2 / n} and q j = (q^2 + j^2 - (q-j)^2)/2,
//     H[q] = s * w_q * sum_j (f_j w_j) conj(w_{q-j}),
// a linear convolution evaluated with FFTs of size M >= max(16, 2n-1): a
// forward FFT of the chirped input, a pointwise product with the FFT of the
// wrapped conjugate chirp b_t = conj(w_t), t in (-n, n) (one table per ring,
// built with the plan), and an inverse FFT.  Synthesis is
// conj(analysis(conj(H))) without the 1/n.  Chirp phases are reduced exactly
// as (t^2 mod 2n)/n.
//
// FFT: Stockham autosort passes of radix 16 (one final pass of radix 2, 4 or
// 8 when log2 M is not a multiple of 4).  Each FFT is owned by T = M/16
// threads holding 16 points each in registers: thread t owns points
// t + i T, i = 0..15, both at the start of the forward FFT and at the end of
// every FFT, so the chirp products, the pointwise product between the two
// FFTs and the output stores need no LDS.  The passes in between exchange
// through LDS (padded by one point per 16 against bank conflicts).  Pass
// (Ns, R) maps butterfly j, inputs x[j + r M/R], to outputs
// y[(j / Ns) Ns R + j % Ns + r Ns] after twiddles w^r,
// w = e^{-+2 pi i (j % Ns)/(Ns R)}: the powers w^(2^b) are read from an
// e^{-2 pi i e/Mmax} table one pass ahead (so the loads overlap the LDS
// exchange) and w^r is their product over the bits of r.  The inverse FFT
// runs the forward's passes with conjugate twiddles.
//
// Work: the rings sharing M form a size class; one launch per direction
// runs every class up to 4096 points (8192-point classes launch on their
// own).  A workgroup runs F = blockDim/T FFTs, one per (ring, map) pair of
// its class; pairs are
// map-fastest so a workgroup's maps share the ring, and workgroup ids are
// remapped so that consecutive pairs stay on one XCD (one L2) -- the map
// -fastest bin array H[(k^2 + q) B + b] is then written by nearby pairs.

#include <algorithm>
#include <array>
#include <type_traits>

#include "common.hpp"

namespace osht {

namespace {

// 16-byte aligned, so that LDS exchanges use 128-bit accesses: with 64-bit
// halves, a 16-byte lane stride puts two lanes of a 16-lane group on each
// bank pair.
struct alignas(16) cplx {
  double x, y;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cplx cconj(cplx a) { return {a.x, -a.y}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.x - b.x, a.y - b.y}; }

constexpr int RPT = 16;  // points per thread
// M >= 2n - 1 with M even gives n <= M/2: the points t + i T with
// i >= RH = RPT/2 lie at or past M/2 and so past every ring of the class.
// They enter the first FFT as zeros and leave the last one unread, so no
// load, chirp product or store touches them.
constexpr int RH = RPT / 2;

// e^{-2 pi i j/16} (forward); the inverse uses the conjugate.
__device__ __forceinline__ cplx w16(int j, bool inv) {
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, h = 0.70710678118654752440;
  const double cs[16] = {1.0, c1, h, s1, 0.0, -s1, -h, -c1, -1.0, -c1, -h, -s1, 0.0, s1, h, c1};
  const double sn[16] = {0.0, -s1, -h, -c1, -1.0, -c1, -h, -s1, 0.0, s1, h, c1, 1.0, c1, h, s1};
  return {cs[j], inv ? -sn[j] : sn[j]};
}

// v * e^{-+2 pi i j/16} with the exact cases spelled out.
template <int J, bool INV>
__device__ __forceinline__ cplx rot16(cplx v) {
  if constexpr (J == 0) return v;
  else if constexpr (J == 4) return INV ? cplx{-v.y, v.x} : cplx{v.y, -v.x};
  else if constexpr (J == 8) return {-v.x, -v.y};
  else if constexpr (J == 12) return INV ? cplx{v.y, -v.x} : cplx{-v.y, v.x};
  else return cmul(v, w16(J, INV));
}

// In-register natural-order DFT of size R on x[0], x[S], ..., x[(R-1) S].
template <int R, int S, bool INV>
struct Dft {
  template <int K>
  static __device__ __forceinline__ void combine(cplx* x, const cplx* e, const cplx* o) {
    if constexpr (K < R / 2) {
      const cplx t = rot16<K * (16 / R), INV>(o[K]);
      x[K * S] = cadd(e[K], t);
      x[(K + R / 2) * S] = csub(e[K], t);
      combine<K + 1>(x, e, o);
    }
  }
  static __device__ __forceinline__ void run(cplx* x) {
    if constexpr (R == 1) {
      return;
    } else if constexpr (R == 2) {
      const cplx a = x[0], b = x[S];
      x[0] = cadd(a, b);
      x[S] = csub(a, b);
    } else {
      cplx e[R / 2], o[R / 2];
#pragma unroll
      for (int i = 0; i < R / 2; ++i) {
        e[i] = x[2 * i * S];
        o[i] = x[(2 * i + 1) * S];
      }
      Dft<R / 2, 1, INV>::run(e);
      Dft<R / 2, 1, INV>::run(o);
      combine<0>(x, e, o);
    }
  }
};

struct FftCtx {
  cplx* lds;        // this FFT's LDS region (M + M/16 points)
  const cplx* tw;   // e^{-2 pi i e / Mmax}
  int logM, logMmax, t, T;
};

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// The radix of pass p of an FFT of size 2^logM: 16, ..., 16, then 2, 4 or 8
// when logM is not a multiple of 4.  Both directions run the same passes
// (the inverse with conjugate twiddles), so pass p always follows 16^p
// points of the transform: Ns = 16^p.
constexpr int pass_radix(int logM, int p) { return p < (logM >> 2) ? 16 : (1 << (logM & 3)); }
constexpr int num_passes(int logM) { return (logM + 3) >> 2; }
constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }
// Base twiddles w, w^2, w^4, w^8 (log2 R of them) per butterfly of pass p > 0.
constexpr int pass_ntw(int logM, int p) {
  return p == 0 ? 1 : (RPT / pass_radix(logM, p)) * ilog2(pass_radix(logM, p));
}

// Loads pass P's base twiddles into pb[c log2(R) + b] = w_c^(2^b), w_c the
// twiddle e^{-2 pi i e / (Ns R)} of butterfly c (e = its index mod Ns).
template <int LOGM, int P>
__device__ __forceinline__ void load_twiddles(cplx* pb, const FftCtx& cx) {
  constexpr int R = pass_radix(LOGM, P), NB = RPT / R, LB = ilog2(R);
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int e = (cx.t + c * cx.T) & ((1 << (4 * P)) - 1);
    const int E = e << (cx.logMmax - 4 * P - LB);  // tw[E] = e^{-2 pi i e / (Ns R)}
#pragma unroll
    for (int b = 0; b < LB; ++b) pb[c * LB + b] = cx.tw[E << b];
  }
}

// One Stockham pass of radix R over the thread's 16 points, held as
// butterflies c = 0..16/R-1 with element r of butterfly c in v[c + r (16/R)].
// TW: multiply input r of each butterfly by w^r first, w^r the product of
// the base twiddles pb[b] = w^(2^b) over the set bits b of r (ascending).
template <int R, bool INV, bool TW>
__device__ __forceinline__ void pass_compute(cplx* v, const cplx* pb) {
  constexpr int NB = RPT / R, LB = ilog2(R);
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if constexpr (TW) {
      cplx p[LB];
#pragma unroll
      for (int b = 0; b < LB; ++b) {
        p[b] = pb[c * LB + b];
        if (INV) p[b].y = -p[b].y;
      }
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cplx w;
        bool have = false;
#pragma unroll
        for (int b = 0; b < LB; ++b) {
          if (r & (1 << b)) {
            w = have ? cmul(w, p[b]) : p[b];
            have = true;
          }
        }
        v[c + r * NB] = cmul(v[c + r * NB], w);
      }
    }
    Dft<R, NB, INV>::run(v + c);
  }
}

template <int R>
__device__ __forceinline__ void pass_store(const cplx* v, const FftCtx& cx, int Ns) {
  constexpr int NB = RPT / R;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int j = cx.t + c * cx.T;
    const int base = (j / Ns) * Ns * R + (j & (Ns - 1));
#pragma unroll
    for (int r = 0; r < R; ++r) cx.lds[pad(base + r * Ns)] = v[c + r * NB];
  }
}

template <int R>
__device__ __forceinline__ void pass_load(cplx* v, const FftCtx& cx) {
  constexpr int NB = RPT / R;
  const int M = 1 << cx.logM;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int j = cx.t + c * cx.T;
#pragma unroll
    for (int r = 0; r < R; ++r) v[c + r * NB] = cx.lds[pad(j + r * (M / R))];
  }
}

// Pass P of an FFT of size 2^LOGM; pb holds its base twiddles (P > 0).
// The next pass's twiddles are loaded right after this pass's arithmetic,
// so they arrive while the barriers and the LDS exchange run.
template <bool INV, int LOGM, int P>
struct FftPass {
  static constexpr int NP = num_passes(LOGM);
  static constexpr int R = pass_radix(LOGM, P);
  static __device__ __forceinline__ void run(cplx* v, const FftCtx& cx, const cplx* pb) {
    if constexpr (P > 0) {
      __syncthreads();  // previous pass's stores visible
      pass_load<R>(v, cx);
      pass_compute<R, INV, true>(v, pb);
    } else {
      pass_compute<R, INV, false>(v, nullptr);
    }
    if constexpr (P < NP - 1) {
      cplx pn[pass_ntw(LOGM, P + 1)];
      load_twiddles<LOGM, P + 1>(pn, cx);
      __syncthreads();  // all loads of this pass done before stores (in place)
      pass_store<R>(v, cx, 1 << (4 * P));
      FftPass<INV, LOGM, P + 1>::run(v, cx, pn);
    }
  }
};

// Full FFT of size M = 2^LOGM (LOGM >= 4), points t + i T in v on entry and
// exit (natural order); the inverse (INV) is the same passes with conjugate
// twiddles, unscaled.  Every thread of the workgroup must call it (it
// contains barriers).
template <bool INV, int LOGM>
__device__ __forceinline__ void fft(cplx* v, const FftCtx& cx) {
  FftPass<INV, LOGM, 0>::run(v, cx, nullptr);
}

// Workgroup -> pair block, keeping consecutive pair blocks on one XCD
// (workgroups are dispatched round-robin over 8 XCDs).
__device__ __forceinline__ int xcd_remap(int bid, int G) {
  const int q = G >> 3, r = G & 7, x = bid & 7, l = bid >> 3;
  return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

struct PairCtx {
  int k, b, n;
  int64_t base, off;
  bool active;
};

// bid, G: the workgroup's index among the G workgroups of its size class
__device__ __forceinline__ PairCtx pair_of(const RingDesc* __restrict__ rings, int k0, int npairs, int B, int T, int bid,
                                           int G) {
  const int F = blockDim.x / T;
  const int pair = xcd_remap(bid, G) * F + (int)(threadIdx.x / T);
  PairCtx pc;
  pc.active = pair < npairs;
  const int pp = pc.active ? pair : 0;
  pc.k = k0 + pp / B;
  pc.b = pp % B;
  const RingDesc r = rings[pc.k];
  pc.n = r.n;
  pc.off = r.off;
  pc.base = (int64_t)pc.k * pc.k;
  return pc;
}

extern __shared__ cplx lds_buf[];

// Builds the FFT of the wrapped conjugate chirp for every ring of one size
// class: b_t = conj(w_t) for |t| < n (t < 0 stored at M + t), zero elsewhere.
template <int LOGM>
__global__ __launch_bounds__(LOGM == 13 ? 512 : 256) void chirp_kernel(const RingDesc* __restrict__ rings, int k0,
                                                                       int nrings, const cplx* __restrict__ chirp_tab,
                                                                       cplx* __restrict__ table,
                                                                       const cplx* __restrict__ tw, int logMmax) {
  constexpr int logM = LOGM, M = 1 << LOGM, T = M / RPT;
  const PairCtx pc = pair_of(rings, k0, nrings, 1, T, blockIdx.x, gridDim.x);
  const int t = threadIdx.x % T;
  FftCtx cx{lds_buf + (threadIdx.x / T) * (M + M / 16), tw, logM, logMmax, t, T};
  const cplx* w = chirp_tab + pc.base;
  cplx v[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int p = t + i * T;
    cplx b = {0.0, 0.0};
    if (pc.active) {
      if (p < pc.n) b = cconj(w[p]);
      else if (p > M - pc.n) b = cconj(w[M - p]);
    }
    v[i] = b;
  }
  fft<false, LOGM>(v, cx);
  if (pc.active) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) table[pc.off + t + i * T] = v[i];
  }
}

// Shared middle of analysis and synthesis: v holds the chirped input at
// points t + i T (zero for i >= RH); on return v holds the unscaled
// convolution at the same points and wo[i], i < RH, the output chirp w_q
// (q = t + i T < n, else 0).
// BATCH: the chirp-spectrum and output-chirp loads are issued together and
// selected after (a load under a branch is waited for before the next one
// is issued; cf of an inactive pair is its ring's, and positions past the
// ring load its last chirp value).  Measured per direction at L = 1024,
// B = 16, with the input loads batched as well: analysis 391 -> 385 us with
// it, synthesis 370 -> 378 us (its registers spill), so only the analysis
// batches them.  The two directions together went 0.80 -> 0.76 ms.  With the
// upper half of each thread's points left out of the loads and stores
// (RH), neither direction spills; batching the synthesis then gains
// nothing (347 us either way) and moves its rounding, so it stays unbatched.
template <int LOGM, bool BATCH>
__device__ __forceinline__ void bluestein(cplx* v, cplx* wo, const FftCtx& cx, const cplx* __restrict__ cf,
                                          const cplx* __restrict__ w, int n, bool active) {
  fft<false, LOGM>(v, cx);
  if constexpr (BATCH) {
    cplx c[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) c[i] = cf[cx.t + i * cx.T];
#pragma unroll
    for (int i = 0; i < RPT; ++i) v[i] = cmul(v[i], active ? c[i] : cplx{0.0, 0.0});
  } else {
#pragma unroll
    for (int i = 0; i < RPT; ++i) v[i] = cmul(v[i], active ? cf[cx.t + i * cx.T] : cplx{0.0, 0.0});
  }
  fft<true, LOGM>(v, cx);
  if constexpr (BATCH) {
#pragma unroll
    for (int i = 0; i < RH; ++i) wo[i] = w[min(cx.t + i * cx.T, n - 1)];
#pragma unroll
    for (int i = 0; i < RH; ++i)
      if (!(active && cx.t + i * cx.T < n)) wo[i] = cplx{0.0, 0.0};
  } else {
#pragma unroll
    for (int i = 0; i < RH; ++i) {
      const int q = cx.t + i * cx.T;
      wo[i] = (active && q < n) ? w[q] : cplx{0.0, 0.0};
    }
  }
}

struct RingArgs {
  const RingDesc* rings;
  const cplx* chirp_fft;
  const cplx* chirp_tab;
  const cplx* tw;
  int logMmax, L, B, flag;  // flag: analysis normalises by 1/n, synthesis scales its input by 1/n
  const cplx* in;           // f (analysis) or H (synthesis)
  cplx* out;                // H (analysis) or f (synthesis)
  double* freal;            // real-map samples (REAL variants)
  int Breal;
};

// Size classes of one ring-DFT launch: workgroups [blk0[c], blk0[c] + nblk[c])
// run the np[c] (ring, map) pairs of rings k0[c].. with FFT size 2^logM[c].
// Every class starts at a multiple of 8 workgroups, so that its local
// workgroup index keeps the XCD round-robin of the global one.
constexpr int kMaxClasses = 12;
struct ClassTab {
  int n;
  int blk0[kMaxClasses], nblk[kMaxClasses], k0[kMaxClasses], np[kMaxClasses], logM[kMaxClasses];
};

// samples f[b][L^2] -> bins H[(k^2 + q) * B + b] (scale 1/n or 1).
template <int LOGM, bool REAL>
__device__ __forceinline__ void analysis_body(const RingArgs& a, int k0, int npairs, int bid, int G) {
  constexpr int logM = LOGM, M = 1 << LOGM, T = M / RPT;
  if (xcd_remap(bid, G) * (int)(blockDim.x / T) >= npairs) return;  // a padding workgroup (uniform)
  const RingDesc* __restrict__ rings = a.rings;
  const cplx* __restrict__ chirp_fft = a.chirp_fft;
  const cplx* __restrict__ chirp_tab = a.chirp_tab;
  const cplx* __restrict__ tw = a.tw;
  const cplx* __restrict__ f = a.in;
  cplx* __restrict__ H = a.out;
  const double* __restrict__ freal = a.freal;
  const int logMmax = a.logMmax, L = a.L, B = a.B, normalise = a.flag, Breal = a.Breal;
  const PairCtx pc = pair_of(rings, k0, npairs, B, T, bid, G);
  const int t = threadIdx.x % T;
  FftCtx cx{lds_buf + (threadIdx.x / T) * (M + M / 16), tw, logM, logMmax, t, T};
  const cplx* w = chirp_tab + pc.base;
  const cplx* fr = f + (int64_t)pc.b * L * L + pc.base;
  // REAL: complex map b carries the real maps 2b (real part) and 2b+1
  const double* fa = freal + (int64_t)(2 * pc.b) * L * L + pc.base;
  const double* fb = fa + (int64_t)L * L;
  const bool has_b = 2 * pc.b + 1 < Breal;
  const double* fbs = has_b ? fb : fa;  // a missing second real map reads the first and drops it
  cplx v[RPT], ws[RH];
  // every load issued before any is used: positions past the ring (and
  // every position of an inactive pair, whose ring is k0) load the ring's
  // last sample, which the select drops
#pragma unroll
  for (int i = 0; i < RH; ++i) {
    const int p = min(t + i * T, pc.n - 1);
    if constexpr (REAL) v[i] = cplx{fa[p], fbs[p]};
    else v[i] = fr[p];
    ws[i] = w[p];
  }
#pragma unroll
  for (int i = 0; i < RH; ++i) {
    cplx x = v[i];
    if constexpr (REAL) {
      if (!has_b) x.y = 0.0;
    }
    v[i] = (pc.active && t + i * T < pc.n) ? cmul(x, ws[i]) : cplx{0.0, 0.0};
  }
#pragma unroll
  for (int i = RH; i < RPT; ++i) v[i] = cplx{0.0, 0.0};
  cplx wo[RH];
  bluestein<LOGM, true>(v, wo, cx, chirp_fft + pc.off, w, pc.n, pc.active);
  if (pc.active) {
    const double sc = (normalise ? 1.0 / pc.n : 1.0) / M;
    cplx* Ht = H + (pc.base + t) * B + pc.b;
    const int64_t hs = (int64_t)T * B;
#pragma unroll
    for (int i = 0; i < RH; ++i) {
      const int q = t + i * T;
      if (q < pc.n) {
        const cplx c = cmul(v[i], wo[i]);
        Ht[i * hs] = {c.x * sc, c.y * sc};
      }
    }
  }
}

// Fold of the inverse transform's per-order values into ring bins:
//   H[(k^2 + q) B + b] = sum_{m = q mod n_k, |m| < L} G'_m(theta_k),
//   G'_m(theta_k) = Y[slot(m)][k][col(m, b)] (complex, two doubles).
// Spin 0: slot(m) = |m|, col = (m < 0 ? 2B : 0) + 2b;  spin != 0:
// slot(m) = m + L - 1, col = 2b.  One workgroup per ring; outputs are
// map-fastest so that each (order, ring) row of Y is read as one contiguous
// vector.  When the ring has fewer outputs than threads, each bin's order
// list is split into C contiguous chunks whose partial sums are added in
// chunk order (fixed summation order, deterministic).
// YT: double, or float for the FP32 inverse apply's output.
// ring_cut[k] (null: L): only orders |m| < ring_cut[k] reach ring k above
// 2^-80 (the rows of the others are neither read nor, on int8 plans,
// written).
template <class YT, int NT>
__global__ __launch_bounds__(NT) void fold_kernel(const YT* __restrict__ Y, cplx* __restrict__ H,
                                                  const int32_t* __restrict__ ring_cut, int L, int B, int spin0,
                                                  int ncols) {
  typedef typename std::conditional<std::is_same<YT, float>::value, float2, double2>::type YT2;
  __shared__ cplx part[NT];
  const int k = blockIdx.x, n = 2 * k + 1;
  const int units = n * B;
  const int C = max(1, NT / units);
  const int64_t base = (int64_t)k * k;
  const int cut = ring_cut ? ring_cut[k] : L;  // 1 <= cut <= L
  for (int u = threadIdx.x; u < units * C; u += NT) {
    const int c = u / units, rem = u - c * units;
    const int q = rem / B, b = rem - q * B;
    const int mstart = q - ((q + cut - 1) / n) * n;  // smallest m > -cut congruent to q
    const int cnt = mstart <= cut - 1 ? (cut - 1 - mstart) / n + 1 : 0;
    const int i0 = (int)((int64_t)cnt * c / C), i1 = (int)((int64_t)cnt * (c + 1) / C);
    cplx h = {0.0, 0.0};
    for (int i = i0; i < i1; ++i) {
      const int m = mstart + i * n;
      int slot, col;
      if (spin0) { slot = m < 0 ? -m : m; col = (m < 0 ? 2 * B : 0) + 2 * b; }
      else { slot = m + L - 1; col = 2 * b; }
      // (re, im) of one column pair: 16 (or 8) aligned bytes, ncols and col even
      const YT2 y = *reinterpret_cast<const YT2*>(Y + ((int64_t)slot * L + k) * ncols + col);
      h.x += (double)y.x;
      h.y += (double)y.y;
    }
    if (C == 1) H[(base + q) * B + b] = h;
    else part[u] = h;
  }
  if (C > 1) {
    __syncthreads();
    for (int u = threadIdx.x; u < units; u += NT) {
      cplx h = part[u];
      for (int c = 1; c < C; ++c) h = cadd(h, part[c * units + u]);
      const int q = u / B, b = u - q * B;
      H[(base + q) * B + b] = h;
    }
  }
}

// Synthesis of (ring, map) pairs from the map-fastest bins H (optionally
// times 1/n): f[b][k^2 + j] = sum_q H_k[q] e^{+2 pi i q j / n}.
template <int LOGM, bool REAL>
__device__ __forceinline__ void synthesis_body(const RingArgs& a, int k0, int npairs, int bid, int G) {
  constexpr int logM = LOGM, M = 1 << LOGM, T = M / RPT;
  if (xcd_remap(bid, G) * (int)(blockDim.x / T) >= npairs) return;  // a padding workgroup (uniform)
  const RingDesc* __restrict__ rings = a.rings;
  const cplx* __restrict__ chirp_fft = a.chirp_fft;
  const cplx* __restrict__ chirp_tab = a.chirp_tab;
  const cplx* __restrict__ tw = a.tw;
  const cplx* __restrict__ H = a.in;
  cplx* __restrict__ f = a.out;
  double* __restrict__ freal = a.freal;
  const int logMmax = a.logMmax, L = a.L, B = a.B, scale_inv_n = a.flag, Breal = a.Breal;
  const PairCtx pc = pair_of(rings, k0, npairs, B, T, bid, G);
  const int t = threadIdx.x % T;
  FftCtx cx{lds_buf + (threadIdx.x / T) * (M + M / 16), tw, logM, logMmax, t, T};
  const cplx* w = chirp_tab + pc.base;
  cplx v[RPT], ws[RH];
  // loads first (clamped to the ring's last bin), selects after
#pragma unroll
  for (int i = 0; i < RH; ++i) {
    const int q = min(t + i * T, pc.n - 1);
    v[i] = H[(pc.base + q) * B + pc.b];
    ws[i] = w[q];
  }
#pragma unroll
  for (int i = RH; i < RPT; ++i) v[i] = cplx{0.0, 0.0};
#pragma unroll
  for (int i = 0; i < RH; ++i) {
    cplx h = {0.0, 0.0};
    if (pc.active && t + i * T < pc.n) {
      h = v[i];
      if (scale_inv_n) { h.x /= pc.n; h.y /= pc.n; }
      h = cmul(cconj(h), ws[i]);
    }
    v[i] = h;
  }
  cplx wo[RH];
  bluestein<LOGM, false>(v, wo, cx, chirp_fft + pc.off, w, pc.n, pc.active);
  if (pc.active) {
    const double sc = 1.0 / M;
    cplx* fr = f + (int64_t)pc.b * L * L + pc.base;
    // REAL: the real part is real map 2b, the imaginary part real map 2b+1
    double* fa = freal + (int64_t)(2 * pc.b) * L * L + pc.base;
    double* fb = fa + (int64_t)L * L;
    const bool has_b = 2 * pc.b + 1 < Breal;
#pragma unroll
    for (int i = 0; i < RH; ++i) {
      const int j = t + i * T;
      if (j < pc.n) {
        const cplx c = cmul(v[i], wo[i]);
        if constexpr (REAL) {
          fa[j] = c.x * sc;
          if (has_b) fb[j] = -c.y * sc;
        } else {
          fr[j] = {c.x * sc, -c.y * sc};
        }
      }
    }
  }
}

// Every size class of one direction in one launch of 256-thread workgroups
// (FFT sizes up to 4096; the largest classes first, so the small ones fill
// the tail): one launch instead of one per class, whose fixed cost
// dominated the small classes.
template <bool SYN, bool REAL>
__global__ __launch_bounds__(256, 2) void ring_dft_multi_kernel(RingArgs a, ClassTab ct) {
  int c = 0;
  while (c + 1 < ct.n && (int)blockIdx.x >= ct.blk0[c + 1]) ++c;
  const int bid = (int)blockIdx.x - ct.blk0[c], G = ct.nblk[c];
  auto run = [&](auto lg) {
    constexpr int LG = decltype(lg)::value;
    if constexpr (SYN) synthesis_body<LG, REAL>(a, ct.k0[c], ct.np[c], bid, G);
    else analysis_body<LG, REAL>(a, ct.k0[c], ct.np[c], bid, G);
  };
  switch (ct.logM[c]) {
    case 4: run(std::integral_constant<int, 4>{}); break;
    case 5: run(std::integral_constant<int, 5>{}); break;
    case 6: run(std::integral_constant<int, 6>{}); break;
    case 7: run(std::integral_constant<int, 7>{}); break;
    case 8: run(std::integral_constant<int, 8>{}); break;
    case 9: run(std::integral_constant<int, 9>{}); break;
    case 10: run(std::integral_constant<int, 10>{}); break;
    case 11: run(std::integral_constant<int, 11>{}); break;
    case 12: run(std::integral_constant<int, 12>{}); break;
    default: break;
  }
}

// 8192-point classes (L > 2048) take 512-thread workgroups of their own.
template <bool SYN, bool REAL>
__global__ __launch_bounds__(512) void ring_dft_8192_kernel(RingArgs a, int k0, int npairs) {
  if constexpr (SYN) synthesis_body<13, REAL>(a, k0, npairs, blockIdx.x, gridDim.x);
  else analysis_body<13, REAL>(a, k0, npairs, blockIdx.x, gridDim.x);
}

// tw[e] = e^{-2 pi i e / Mmax}; chirp_tab[k^2 + t] = e^{-i pi (t^2 mod 2n)/n},
// n = 2k+1, t < n.
__global__ void table_kernel(cplx* tw, int Mmax, cplx* chirp_tab, int L) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double s, c;
  if (i < Mmax) {
    sincospi(-2.0 * (double)i / (double)Mmax, &s, &c);
    tw[i] = {c, s};
  }
  if (i < (int64_t)L * L) {
    int k = (int)sqrt((double)i);
    while ((int64_t)(k + 1) * (k + 1) <= i) ++k;
    while ((int64_t)k * k > i) --k;
    const int64_t t = i - (int64_t)k * k, n = 2 * k + 1;
    const int64_t rr = (t * t) % (2 * n);
    sincospi(-(double)rr / (double)n, &s, &c);
    chirp_tab[i] = {c, s};
  }
}

// Launch shape of a size class: threads per workgroup and pairs per workgroup.
struct Shape {
  int nthr, F;
  size_t lds;
};

Shape shape_for(int logM) {
  const int T = (1 << logM) / RPT;
  const int nthr = std::max(T, 256);
  const int F = nthr / T;
  const size_t per = (size_t)(1 << logM) + ((1 << logM) >> 4);
  // a 16-point FFT stays in registers
  const size_t lds = logM > 4 ? sizeof(cplx) * per * F : 0;
  return Shape{nthr, F, lds};
}

void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 65536) OSHT_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

// Calls fn(std::integral_constant<int, logM>) for logM in [4, 13].
template <class Fn>
void with_logM(int logM, Fn fn) {
  switch (logM) {
    case 4: fn(std::integral_constant<int, 4>{}); break;
    case 5: fn(std::integral_constant<int, 5>{}); break;
    case 6: fn(std::integral_constant<int, 6>{}); break;
    case 7: fn(std::integral_constant<int, 7>{}); break;
    case 8: fn(std::integral_constant<int, 8>{}); break;
    case 9: fn(std::integral_constant<int, 9>{}); break;
    case 10: fn(std::integral_constant<int, 10>{}); break;
    case 11: fn(std::integral_constant<int, 11>{}); break;
    case 12: fn(std::integral_constant<int, 12>{}); break;
    case 13: fn(std::integral_constant<int, 13>{}); break;
    default: throw Error{OSHT_ENOTSUP, "ring FFT size out of range"};
  }
}

// Size classes: contiguous ring ranges [k_lo, k_hi) sharing logM.
template <class Fn>
void for_each_class(const Plan& p, Fn fn) {
  int k = 0;
  while (k < p.L) {
    const int logM = p.h_ring_logM[k];
    int e = k;
    while (e < p.L && p.h_ring_logM[e] == logM) ++e;
    fn(k, e, logM);
    k = e;
  }
}

}  // namespace

void build_chirps(Plan& p) {
  const int L = p.L;
  std::vector<RingDesc> rings(L);
  int64_t off = 0;
  int maxlog = 4;
  p.h_ring_logM.assign(L, 0);
  for (int k = 0; k < L; ++k) {
    const int n = 2 * k + 1;
    int logM = 4;
    while ((1 << logM) < 2 * n - 1) ++logM;
    rings[k] = RingDesc{n, logM, off};
    p.h_ring_logM[k] = logM;
    off += (int64_t)1 << logM;
    maxlog = std::max(maxlog, logM);
  }
  OSHT_CHECK(maxlog <= 13, OSHT_ENOTSUP, "ring FFTs above 8192 points are not supported");
  p.max_logM = maxlog;
  upload(p.d_rings, rings);
  const int Mmax = 1 << p.max_logM;
  p.d_twiddle.alloc(sizeof(cplx) * Mmax);
  p.d_chirp_tab.alloc(sizeof(cplx) * (size_t)L * L);
  const int64_t nthr = std::max<int64_t>((int64_t)L * L, Mmax);
  hipLaunchKernelGGL(table_kernel, dim3((unsigned)ceil_div(nthr, 256)), dim3(256), 0, 0, p.d_twiddle.as<cplx>(), Mmax,
                     p.d_chirp_tab.as<cplx>(), L);
  OSHT_HIP(hipGetLastError());
  p.d_chirp.alloc(sizeof(cplx) * off);
  for_each_class(p, [&](int k0, int k1, int logM) {
    with_logM(logM, [&](auto lg) {
      constexpr int LG = decltype(lg)::value;
      const Shape sh = shape_for(LG);
      allow_lds((const void*)chirp_kernel<LG>, sh.lds);
      const int np = k1 - k0;
      hipLaunchKernelGGL(chirp_kernel<LG>, dim3((unsigned)ceil_div(np, sh.F)), dim3(sh.nthr), sh.lds, 0,
                         p.d_rings.as<RingDesc>(), k0, np, p.d_chirp_tab.as<cplx>(), p.d_chirp.as<cplx>(),
                         p.d_twiddle.as<cplx>(), p.max_logM);
      OSHT_HIP(hipGetLastError());
    });
  });
}

namespace {

// One direction of the ring DFTs: all size classes up to 4096 points in one
// launch (largest first), 8192-point classes in launches of their own.
void launch_ring_dft(const Plan& p, bool syn, const RingArgs& a, int64_t B, hipStream_t st) {
  std::vector<std::array<int, 3>> cls;  // (logM, k0, k1)
  for_each_class(p, [&](int k0, int k1, int logM) { cls.push_back({logM, k0, k1}); });
  std::sort(cls.begin(), cls.end(), [](const std::array<int, 3>& x, const std::array<int, 3>& y) {
    return x[0] > y[0];
  });
  ClassTab ct{};
  int blk = 0;
  size_t lds = 0;
  const bool real = a.Breal > 0;
  for (const auto& c : cls) {
    const int logM = c[0], np = (c[2] - c[1]) * (int)B;
    if (logM == 13) {
      const Shape sh = shape_for(13);
      auto go = [&](auto kernel) {
        allow_lds((const void*)kernel, sh.lds);
        hipLaunchKernelGGL(kernel, dim3((unsigned)ceil_div(np, sh.F)), dim3(sh.nthr), sh.lds, st, a, c[1], np);
        OSHT_HIP(hipGetLastError());
      };
      if (syn) real ? go(ring_dft_8192_kernel<true, true>) : go(ring_dft_8192_kernel<true, false>);
      else real ? go(ring_dft_8192_kernel<false, true>) : go(ring_dft_8192_kernel<false, false>);
      continue;
    }
    OSHT_CHECK(ct.n < kMaxClasses, OSHT_ENOTSUP, "too many ring FFT size classes");
    const Shape sh = shape_for(logM);
    const int nb = (int)ceil_div(ceil_div(np, sh.F), 8) * 8;
    ct.blk0[ct.n] = blk;
    ct.nblk[ct.n] = nb;
    ct.k0[ct.n] = c[1];
    ct.np[ct.n] = np;
    ct.logM[ct.n] = logM;
    ++ct.n;
    blk += nb;
    lds = std::max(lds, sh.lds);
  }
  if (ct.n == 0) return;
  auto go = [&](auto kernel) {
    allow_lds((const void*)kernel, lds);
    hipLaunchKernelGGL(kernel, dim3((unsigned)blk), dim3(256), lds, st, a, ct);
    OSHT_HIP(hipGetLastError());
  };
  if (syn) real ? go(ring_dft_multi_kernel<true, true>) : go(ring_dft_multi_kernel<true, false>);
  else real ? go(ring_dft_multi_kernel<false, true>) : go(ring_dft_multi_kernel<false, false>);
}

}  // namespace

void launch_ring_analysis(const Plan& p, const double* f, double* H, int64_t B, bool normalise, hipStream_t st,
                          int64_t real_maps) {
  const RingArgs a{p.d_rings.as<RingDesc>(), p.d_chirp.as<cplx>(), p.d_chirp_tab.as<cplx>(), p.d_twiddle.as<cplx>(),
                   p.max_logM, p.L, (int)B, normalise ? 1 : 0, reinterpret_cast<const cplx*>(f),
                   reinterpret_cast<cplx*>(H), const_cast<double*>(f), (int)real_maps};
  launch_ring_dft(p, false, a, B, st);
}

// 1024 threads per ring: each thread's bins are summed one after another, so
// the thread count sets how many loads are in flight (256 threads: 0.19 ms,
// 1024: 0.16 ms at L = 1024, B = 16; FP32 Y 0.18 -> 0.12 ms).
constexpr int kFoldThreads = 1024;

void launch_fold(const Plan& p, const double* Y, double* H, int64_t B, hipStream_t st) {
  // FP32 plans: the inverse apply wrote its output in FP32
  if (p.fp32)
    hipLaunchKernelGGL((fold_kernel<float, kFoldThreads>), dim3(p.L), dim3(kFoldThreads), 0, st,
                       reinterpret_cast<const float*>(Y), reinterpret_cast<cplx*>(H), p.d_ring_cut.as<int32_t>(), p.L,
                       (int)B, p.spin == 0 ? 1 : 0, p.ncols_per_map * (int)B);
  else
    hipLaunchKernelGGL((fold_kernel<double, kFoldThreads>), dim3(p.L), dim3(kFoldThreads), 0, st, Y,
                       reinterpret_cast<cplx*>(H), p.d_ring_cut.as<int32_t>(), p.L, (int)B, p.spin == 0 ? 1 : 0,
                       p.ncols_per_map * (int)B);
  OSHT_HIP(hipGetLastError());
}

void launch_ring_synthesis(const Plan& p, const double* H, int scale_inv_n, double* f, int64_t B, hipStream_t st,
                           int64_t real_maps) {
  const RingArgs a{p.d_rings.as<RingDesc>(), p.d_chirp.as<cplx>(), p.d_chirp_tab.as<cplx>(), p.d_twiddle.as<cplx>(),
                   p.max_logM, p.L, (int)B, scale_inv_n, reinterpret_cast<const cplx*>(H),
                   reinterpret_cast<cplx*>(f), f, (int)real_maps};
  launch_ring_dft(p, true, a, B, st);
}

}  // namespace osht
