// Ring DFTs of the odd lengths n = 2k+1 (k = 0..L-1) by Bluestein's chirp-z
// algorithm on power-of-two FFTs held in LDS.
//
// Analysis (ring k, one map):      H[q] = s * sum_j f_j e^{-2 pi i q j / n}
// Synthesis:                       f_j  =     sum_q H[q] e^{+2 pi i q j / n}
// With w_t = e^{-i pi t^2 / n} and q j = (q^2 + j^2 - (q-j)^2)/2,
//     H[q] = s * w_q * sum_j (f_j w_j) conj(w_{q-j}),
// a linear convolution evaluated by FFTs of size M >= 2n-1: a forward DIT
// FFT (bit-reversed in, natural out), a pointwise product with the FFT of
// the wrapped conjugate chirp b_t = conj(w_t), t in (-n, n) (computed once
// per plan), and an inverse DIF FFT (natural in, bit-reversed out).
// Synthesis is conj(analysis(conj(H))) without the 1/n.  Chirp phases are
// reduced exactly as (t^2 mod 2n)/n and tabulated per ring at plan time.
//
// FFT passes are radix 4 (two radix-2 stages fused; one radix-2 stage when
// log2 M is odd).  Twiddles e^{-2 pi i j/Mmax} are the product of two small
// tables T1[j >> 6] T2[j & 63] kept in LDS.  Rings are launched by FFT size
// class so that each launch reserves only the LDS its rings need.
//
// Layouts: samples and coefficients of the C ABI are [b][L^2]; ring bins are
// kept map-fastest, H[(k^2 + q) * B + b], which is what the order-wise GEMMs
// read.  One workgroup handles one (ring, map).

#include "common.hpp"

namespace osht {

namespace {

struct cplx {
  double x, y;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cplx cconj(cplx a) { return {a.x, -a.y}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cplx cmul_negi(cplx a) { return {a.y, -a.x}; }  // a * (-i)

__device__ __forceinline__ unsigned bitrev(unsigned v, int bits) {
  return bits == 0 ? 0u : (__brev(v) >> (32 - bits));
}

struct Tw {
  const cplx* t1;  // e^{-2 pi i 64 a / Mmax}
  const cplx* t2;  // e^{-2 pi i c / Mmax}, c < 64
  int shift;       // log2(Mmax / M)
  bool inverse;
  __device__ __forceinline__ cplx operator()(int j) const {  // e^{-+2 pi i j / M}
    const int J = j << shift;
    cplx w = cmul(t1[J >> 6], t2[J & 63]);
    if (inverse) w.y = -w.y;
    return w;
  }
};

// In-place DIT FFT of size M = 2^logM (bit-reversed input, natural output).
__device__ void fft_dit(cplx* x, int logM, const Tw& tw) {
  const int M = 1 << logM;
  int s = 0;  // number of radix-2 stages done
  if (logM & 1) {
    for (int i = threadIdx.x; i < M / 2; i += blockDim.x) {
      const cplx u = x[2 * i], v = x[2 * i + 1];
      x[2 * i] = cadd(u, v);
      x[2 * i + 1] = csub(u, v);
    }
    __syncthreads();
    s = 1;
  }
  for (; s < logM; s += 2) {
    const int h = 1 << s;  // half-size of the first fused stage
    for (int bf = threadIdx.x; bf < M / 4; bf += blockDim.x) {
      const int pos = bf & (h - 1);
      const int base = (bf >> s) << (s + 2);
      cplx* p = x + base + pos;
      const cplx w1 = tw(pos << (logM - s - 1));  // W_{2h}^{pos}
      const cplx w2 = tw(pos << (logM - s - 2));  // W_{4h}^{pos}
      const cplx a0 = p[0], a1 = cmul(w1, p[h]), a2 = p[2 * h], a3 = cmul(w1, p[3 * h]);
      const cplx b0 = cadd(a0, a1), b1 = csub(a0, a1), b2 = cadd(a2, a3), b3 = csub(a2, a3);
      const cplx t2 = cmul(w2, b2);
      cplx t3 = cmul(w2, b3);
      t3 = tw.inverse ? cplx{-t3.y, t3.x} : cmul_negi(t3);  // W_{4h}^{pos+h} = -+i W_{4h}^{pos}
      p[0] = cadd(b0, t2);
      p[2 * h] = csub(b0, t2);
      p[h] = cadd(b1, t3);
      p[3 * h] = csub(b1, t3);
    }
    __syncthreads();
  }
}

// In-place DIF FFT (natural input, bit-reversed output).
__device__ void fft_dif(cplx* x, int logM, const Tw& tw) {
  const int M = 1 << logM;
  int s = logM;  // stages remaining, largest half first
  for (; s >= 2; s -= 2) {
    const int h = 1 << (s - 2);  // pairs (pos, pos+2h) then (pos, pos+h)
    for (int bf = threadIdx.x; bf < M / 4; bf += blockDim.x) {
      const int pos = bf & (h - 1);
      const int base = (bf >> (s - 2)) << s;
      cplx* p = x + base + pos;
      const cplx w2 = tw(pos << (logM - s));      // W_{4h}^{pos}
      const cplx w1 = tw(pos << (logM - s + 1));  // W_{2h}^{pos}
      const cplx a0 = p[0], a1 = p[h], a2 = p[2 * h], a3 = p[3 * h];
      const cplx b0 = cadd(a0, a2), b1 = cadd(a1, a3);
      const cplx b2 = cmul(w2, csub(a0, a2));
      cplx d = csub(a1, a3);
      d = tw.inverse ? cplx{-d.y, d.x} : cmul_negi(d);
      const cplx b3 = cmul(w2, d);
      p[0] = cadd(b0, b1);
      p[h] = cmul(w1, csub(b0, b1));
      p[2 * h] = cadd(b2, b3);
      p[3 * h] = cmul(w1, csub(b2, b3));
    }
    __syncthreads();
  }
  if (s == 1) {
    for (int i = threadIdx.x; i < M / 2; i += blockDim.x) {
      const cplx u = x[2 * i], v = x[2 * i + 1];
      x[2 * i] = cadd(u, v);
      x[2 * i + 1] = csub(u, v);
    }
    __syncthreads();
  }
}

extern __shared__ cplx lds_buf[];

// LDS layout: [0, M) data, then T1 (Mmax/64 entries, at least 1), T2 (64).
__device__ __forceinline__ Tw load_tw(const cplx* __restrict__ g_t1, const cplx* __restrict__ g_t2, int logMmax,
                                      int logM, bool inverse) {
  const int M = 1 << logM;
  const int n1 = max(1, (1 << logMmax) >> 6);
  cplx* t1 = lds_buf + M;
  cplx* t2 = t1 + n1;
  for (int i = threadIdx.x; i < n1; i += blockDim.x) t1[i] = g_t1[i];
  for (int i = threadIdx.x; i < 64; i += blockDim.x) t2[i] = g_t2[i];
  return Tw{t1, t2, logMmax - logM, inverse};
}

// Builds the FFT of the wrapped conjugate chirp for every ring of one size
// class (rings k0 .. k0 + gridDim.x - 1).
__global__ void chirp_kernel(const RingDesc* __restrict__ rings, int k0, const cplx* __restrict__ chirp_tab,
                             cplx* __restrict__ table, const cplx* __restrict__ g_t1, const cplx* __restrict__ g_t2,
                             int logMmax) {
  const int k = k0 + blockIdx.x;
  const RingDesc r = rings[k];
  const int M = 1 << r.logM, n = r.n;
  const Tw tw = load_tw(g_t1, g_t2, logMmax, r.logM, false);
  cplx* x = lds_buf;
  for (int i = threadIdx.x; i < M; i += blockDim.x) x[i] = {0.0, 0.0};
  __syncthreads();
  const cplx* w = chirp_tab + (int64_t)k * k;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const cplx b = cconj(w[t]);
    x[bitrev(t, r.logM)] = b;
    if (t > 0) x[bitrev(M - t, r.logM)] = b;
  }
  __syncthreads();
  fft_dit(x, r.logM, tw);
  for (int i = threadIdx.x; i < M; i += blockDim.x) table[r.off + i] = x[i];
}

// Bluestein core: a_j (already times w_j) at bit-reversed positions of x,
// zero elsewhere; leaves conv[q] at position bitrev(q), unscaled by 1/M.
__device__ void bluestein_core(cplx* x, const RingDesc& r, const cplx* __restrict__ chirp_fft, const Tw& fwd,
                               const Tw& inv) {
  const int M = 1 << r.logM;
  fft_dit(x, r.logM, fwd);
  for (int i = threadIdx.x; i < M; i += blockDim.x) x[i] = cmul(x[i], chirp_fft[r.off + i]);
  __syncthreads();
  fft_dif(x, r.logM, inv);
}

// samples f[b][L^2] -> bins H[(k^2 + q) * B + b] (scale s = 1/n or 1).
__global__ void ring_analysis_kernel(const RingDesc* __restrict__ rings, int k0, const cplx* __restrict__ chirp_fft,
                                     const cplx* __restrict__ chirp_tab, const cplx* __restrict__ g_t1,
                                     const cplx* __restrict__ g_t2, int logMmax, int L, const cplx* __restrict__ f,
                                     cplx* __restrict__ H, int B, int normalise) {
  const int k = k0 + blockIdx.x, b = blockIdx.y;
  const RingDesc r = rings[k];
  const int M = 1 << r.logM, n = r.n;
  const int64_t base = (int64_t)k * k;
  const Tw fwd = load_tw(g_t1, g_t2, logMmax, r.logM, false);
  Tw inv = fwd;
  inv.inverse = true;
  cplx* x = lds_buf;
  const cplx* w = chirp_tab + base;
  for (int i = threadIdx.x; i < M; i += blockDim.x) x[i] = {0.0, 0.0};
  __syncthreads();
  const cplx* fr = f + (int64_t)b * L * L + base;
  for (int j = threadIdx.x; j < n; j += blockDim.x) x[bitrev(j, r.logM)] = cmul(fr[j], w[j]);
  __syncthreads();
  bluestein_core(x, r, chirp_fft, fwd, inv);
  const double sc = (normalise ? 1.0 / n : 1.0) / M;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const cplx c = cmul(x[bitrev(q, r.logM)], w[q]);
    H[(base + q) * B + b] = {c.x * sc, c.y * sc};
  }
}

// Synthesis of ring k, map b, with the bins taken either from the
// map-fastest bin array H (optionally times 1/n), or folded from the
// per-order GEMM output Y of the inverse transform:
//   H[q] = sum_{m = q mod n, |m| < L} G'_m(theta_k),
//   G'_m(theta_k) = Y[slot(m)][k][col(m, b)] (complex, two doubles).
// Spin 0: slot(m) = |m|, col = (m < 0 ? 2B : 0) + 2b;  spin != 0:
// slot(m) = m + L - 1, col = 2b.  Summation order is fixed (see the fold).
__global__ void ring_synthesis_kernel(const RingDesc* __restrict__ rings, int k0, const cplx* __restrict__ chirp_fft,
                                      const cplx* __restrict__ chirp_tab, const cplx* __restrict__ g_t1,
                                      const cplx* __restrict__ g_t2, int logMmax, int L, const cplx* __restrict__ H,
                                      int scale_inv_n, const double* __restrict__ Y, int spin0, int ncols,
                                      cplx* __restrict__ f, int B) {
  const int k = k0 + blockIdx.x, b = blockIdx.y;
  const RingDesc r = rings[k];
  const int M = 1 << r.logM, n = r.n;
  const int64_t base = (int64_t)k * k;
  const Tw fwd = load_tw(g_t1, g_t2, logMmax, r.logM, false);
  Tw inv = fwd;
  inv.inverse = true;
  cplx* x = lds_buf;
  const cplx* w = chirp_tab + base;
  for (int i = threadIdx.x; i < M; i += blockDim.x) x[i] = {0.0, 0.0};
  __syncthreads();
  if (Y == nullptr) {
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
      cplx h = H[(base + q) * B + b];
      if (scale_inv_n) { h.x /= n; h.y /= n; }
      x[bitrev(q, r.logM)] = cmul(cconj(h), w[q]);
    }
  } else {
    // Fold: bin q collects the orders m = q (mod n), |m| < L.  When the ring
    // has few bins, each bin's order list is split into C contiguous chunks
    // summed by different threads, then the C partials are added in chunk
    // order (fixed summation order, deterministic).
    const int C = max(1, (int)blockDim.x / n);
    cplx* part = lds_buf + M + max(1, (1 << logMmax) >> 6) + 64;  // C * n <= blockDim.x entries
    for (int t = threadIdx.x; t < n * C; t += blockDim.x) {
      const int q = t % n, c = t / n;
      const int mstart = q - ((q + L - 1) / n) * n;  // smallest m >= -(L-1) congruent to q
      const int cnt = (L - 1 - mstart) / n + 1;
      const int i0 = (int)((int64_t)cnt * c / C), i1 = (int)((int64_t)cnt * (c + 1) / C);
      cplx h = {0.0, 0.0};
      for (int i = i0; i < i1; ++i) {
        const int m = mstart + i * n;
        int slot, col;
        if (spin0) { slot = m < 0 ? -m : m; col = (m < 0 ? 2 * B : 0) + 2 * b; }
        else { slot = m + L - 1; col = 2 * b; }
        const double2 y = *reinterpret_cast<const double2*>(Y + ((int64_t)slot * L + k) * ncols + col);
        h.x += y.x;
        h.y += y.y;
      }
      if (C == 1) x[bitrev(q, r.logM)] = cmul(cconj(h), w[q]);
      else part[c * n + q] = h;
    }
    if (C > 1) {
      __syncthreads();
      for (int q = threadIdx.x; q < n; q += blockDim.x) {
        cplx h = part[q];
        for (int c = 1; c < C; ++c) h = cadd(h, part[c * n + q]);
        x[bitrev(q, r.logM)] = cmul(cconj(h), w[q]);
      }
    }
  }
  __syncthreads();
  bluestein_core(x, r, chirp_fft, fwd, inv);
  const double sc = 1.0 / M;
  cplx* fr = f + (int64_t)b * L * L + base;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const cplx c = cmul(x[bitrev(j, r.logM)], w[j]);
    fr[j] = {c.x * sc, -c.y * sc};
  }
}

// Tables: T1[a] = e^{-2 pi i 64 a / Mmax}, T2[c] = e^{-2 pi i c / Mmax};
// chirp_tab[k^2 + t] = e^{-i pi (t^2 mod 2n)/n}, n = 2k+1, t < n.
__global__ void table_kernel(cplx* t1, cplx* t2, int Mmax, cplx* chirp_tab, int L) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int n1 = max(1, Mmax >> 6);
  double s, c;
  if (i < n1) {
    sincospi(-2.0 * (double)(64 * i) / (double)Mmax, &s, &c);
    t1[i] = {c, s};
  }
  if (i < 64) {
    sincospi(-2.0 * (double)i / (double)Mmax, &s, &c);
    t2[i] = {c, s};
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

void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 65536) OSHT_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

size_t lds_bytes(int logM, int logMmax) {
  return sizeof(cplx) * (((size_t)1 << logM) + std::max(1, (1 << logMmax) >> 6) + 64 + 256);
}

int threads_for(int logM) {
  const int bf = std::max(1, (1 << logM) / 4);
  return bf >= 256 ? 256 : (bf >= 128 ? 128 : 64);
}

// Size classes: contiguous ring ranges [k_lo, k_hi) sharing logM.
template <class F>
void for_each_class(const Plan& p, F fn) {
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
  int maxlog = 0;
  p.h_ring_logM.assign(L, 0);
  for (int k = 0; k < L; ++k) {
    const int n = 2 * k + 1;
    int logM = 0;
    while ((1 << logM) < 2 * n - 1) ++logM;
    rings[k] = RingDesc{n, logM, off};
    p.h_ring_logM[k] = logM;
    off += (int64_t)1 << logM;
    maxlog = std::max(maxlog, logM);
  }
  p.max_logM = std::max(maxlog, 1);
  upload(p.d_rings, rings);
  const int Mmax = 1 << p.max_logM;
  const int n1 = std::max(1, Mmax >> 6);
  p.d_twiddle.alloc(sizeof(cplx) * (n1 + 64));
  p.d_chirp_tab.alloc(sizeof(cplx) * (size_t)L * L);
  cplx* t1 = p.d_twiddle.as<cplx>();
  cplx* t2 = t1 + n1;
  const int64_t nthr = std::max<int64_t>((int64_t)L * L, std::max(n1, 64));
  hipLaunchKernelGGL(table_kernel, dim3((unsigned)ceil_div(nthr, 256)), dim3(256), 0, 0, t1, t2, Mmax,
                     p.d_chirp_tab.as<cplx>(), L);
  OSHT_HIP(hipGetLastError());
  p.d_chirp.alloc(sizeof(cplx) * off);
  for_each_class(p, [&](int k0, int k1, int logM) {
    const size_t lds = lds_bytes(logM, p.max_logM);
    allow_lds((const void*)chirp_kernel, lds);
    hipLaunchKernelGGL(chirp_kernel, dim3(k1 - k0), dim3(threads_for(logM)), lds, 0, p.d_rings.as<RingDesc>(), k0,
                       p.d_chirp_tab.as<cplx>(), p.d_chirp.as<cplx>(), t1, t2, p.max_logM);
    OSHT_HIP(hipGetLastError());
  });
}

void launch_ring_analysis(const Plan& p, const double* f, double* H, int64_t B, bool normalise, hipStream_t st) {
  const int Mmax = 1 << p.max_logM;
  const cplx* t1 = p.d_twiddle.as<cplx>();
  const cplx* t2 = t1 + std::max(1, Mmax >> 6);
  for_each_class(p, [&](int k0, int k1, int logM) {
    const size_t lds = lds_bytes(logM, p.max_logM);
    allow_lds((const void*)ring_analysis_kernel, lds);
    hipLaunchKernelGGL(ring_analysis_kernel, dim3(k1 - k0, (unsigned)B), dim3(threads_for(logM)), lds, st,
                       p.d_rings.as<RingDesc>(), k0, p.d_chirp.as<cplx>(), p.d_chirp_tab.as<cplx>(), t1, t2,
                       p.max_logM, p.L, reinterpret_cast<const cplx*>(f), reinterpret_cast<cplx*>(H), (int)B,
                       normalise ? 1 : 0);
    OSHT_HIP(hipGetLastError());
  });
}

void launch_ring_synthesis(const Plan& p, const double* H, int scale_inv_n, const double* Y, double* f, int64_t B,
                           hipStream_t st) {
  const int Mmax = 1 << p.max_logM;
  const cplx* t1 = p.d_twiddle.as<cplx>();
  const cplx* t2 = t1 + std::max(1, Mmax >> 6);
  for_each_class(p, [&](int k0, int k1, int logM) {
    const size_t lds = lds_bytes(logM, p.max_logM);
    allow_lds((const void*)ring_synthesis_kernel, lds);
    const int nthr = Y ? 256 : threads_for(logM);  // folding small rings wants many threads
    hipLaunchKernelGGL(ring_synthesis_kernel, dim3(k1 - k0, (unsigned)B), dim3(nthr), lds, st,
                       p.d_rings.as<RingDesc>(), k0, p.d_chirp.as<cplx>(), p.d_chirp_tab.as<cplx>(), t1, t2,
                       p.max_logM, p.L, reinterpret_cast<const cplx*>(H), scale_inv_n, Y, p.spin == 0 ? 1 : 0,
                       p.ncols_per_map * (int)B, reinterpret_cast<cplx*>(f), (int)B);
    OSHT_HIP(hipGetLastError());
  });
}

}  // namespace osht
