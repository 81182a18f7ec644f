// Ring DFTs of the odd lengths n = 2k+1 (k = 0..L-1) by Bluestein's chirp-z
// algorithm on power-of-two FFTs held in LDS.
//
// Analysis (ring k, one map):      H[q] = s * sum_j f_j e^{-2 pi i q j / n}
// Synthesis:                       f_j  =     sum_q H[q] e^{+2 pi i q j / n}
// With w_t = e^{-i pi t^2 / n} and q j = (q^2 + j^2 - (q-j)^2)/2,
//     H[q] = s * w_q * sum_j (f_j w_j) conj(w_{q-j}),
// a linear convolution evaluated by FFTs of size M >= 2n-1.  The FFT of the
// chirp b_t = conj(w_t) (t in (-n, n), wrapped modulo M) is computed once per
// plan; synthesis is conj(analysis(conj(H))) without the 1/n.  Chirp phases
// are reduced exactly as (t^2 mod 2n)/n before sincospi.
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

__device__ __forceinline__ unsigned bitrev(unsigned v, int bits) {
  return bits == 0 ? 0u : (__brev(v) >> (32 - bits));
}

// chirp w_t = e^{-i pi (t^2 mod 2n)/n}
__device__ __forceinline__ cplx chirp(int64_t t, int n) {
  const int64_t r = (t * t) % (2 * (int64_t)n);
  double s, c;
  sincospi(-(double)r / (double)n, &s, &c);
  return {c, s};
}

// In-place radix-2 decimation-in-time FFT over x[0..M) (bit-reversed input,
// natural output).  Twiddles tw[j] = e^{-2 pi i j / Mmax}, j < Mmax/2.
// inverse = true conjugates the twiddles (no scaling).
__device__ void fft_dit(cplx* x, int logM, const cplx* __restrict__ tw, int logMmax, bool inverse) {
  const int M = 1 << logM;
  for (int s = 1; s <= logM; ++s) {
    const int half = 1 << (s - 1);
    const int tstride = 1 << (logMmax - s);
    for (int bfly = threadIdx.x; bfly < M / 2; bfly += blockDim.x) {
      const int pos = bfly & (half - 1);
      const int i = ((bfly >> (s - 1)) << s) + pos;
      const int j = i + half;
      cplx w = tw[pos * tstride];
      if (inverse) w.y = -w.y;
      const cplx t = cmul(w, x[j]);
      const cplx u = x[i];
      x[i] = {u.x + t.x, u.y + t.y};
      x[j] = {u.x - t.x, u.y - t.y};
    }
    __syncthreads();
  }
}

// In-place radix-2 decimation-in-frequency FFT (natural input, bit-reversed
// output).
__device__ void fft_dif(cplx* x, int logM, const cplx* __restrict__ tw, int logMmax, bool inverse) {
  const int M = 1 << logM;
  for (int s = logM; s >= 1; --s) {
    const int half = 1 << (s - 1);
    const int tstride = 1 << (logMmax - s);
    for (int bfly = threadIdx.x; bfly < M / 2; bfly += blockDim.x) {
      const int pos = bfly & (half - 1);
      const int i = ((bfly >> (s - 1)) << s) + pos;
      const int j = i + half;
      cplx w = tw[pos * tstride];
      if (inverse) w.y = -w.y;
      const cplx u = x[i], v = x[j];
      x[i] = {u.x + v.x, u.y + v.y};
      x[j] = cmul(w, cplx{u.x - v.x, u.y - v.y});
    }
    __syncthreads();
  }
}

extern __shared__ cplx lds_buf[];

// Builds the FFT of the wrapped conjugate chirp for every ring.
__global__ __launch_bounds__(256) void chirp_kernel(const RingDesc* __restrict__ rings, cplx* __restrict__ table,
                                                    const cplx* __restrict__ tw, int logMmax) {
  const RingDesc r = rings[blockIdx.x];
  const int M = 1 << r.logM, n = r.n;
  cplx* x = lds_buf;
  for (int i = threadIdx.x; i < M; i += blockDim.x) x[i] = {0.0, 0.0};
  __syncthreads();
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const cplx b = cconj(chirp(t, n));
    x[bitrev(t, r.logM)] = b;
    if (t > 0) x[bitrev(M - t, r.logM)] = b;
  }
  __syncthreads();
  fft_dit(x, r.logM, tw, logMmax, false);
  for (int i = threadIdx.x; i < M; i += blockDim.x) table[r.off + i] = x[i];
}

// Core of Bluestein: given a_j already multiplied by w_j and placed at
// bit-reversed positions of x (zero elsewhere), leaves conv[q] at position
// bitrev(q) (unscaled by 1/M).
__device__ void bluestein_core(cplx* x, const RingDesc& r, const cplx* __restrict__ chirp_fft,
                               const cplx* __restrict__ tw, int logMmax) {
  const int M = 1 << r.logM;
  fft_dit(x, r.logM, tw, logMmax, false);
  for (int i = threadIdx.x; i < M; i += blockDim.x) x[i] = cmul(x[i], chirp_fft[r.off + i]);
  __syncthreads();
  fft_dif(x, r.logM, tw, logMmax, true);
}

// samples f[b][L^2] -> bins H[(k^2 + q) * B + b] (scale s = 1/n or 1).
__global__ __launch_bounds__(256) void ring_analysis_kernel(const RingDesc* __restrict__ rings,
                                                            const cplx* __restrict__ chirp_fft,
                                                            const cplx* __restrict__ tw, int logMmax, int L,
                                                            const cplx* __restrict__ f, cplx* __restrict__ H,
                                                            int B, int normalise) {
  const int k = blockIdx.x, b = blockIdx.y;
  const RingDesc r = rings[k];
  const int M = 1 << r.logM, n = r.n;
  const int64_t base = (int64_t)k * k;
  cplx* x = lds_buf;
  for (int i = threadIdx.x; i < M; i += blockDim.x) x[i] = {0.0, 0.0};
  __syncthreads();
  const cplx* fr = f + (int64_t)b * L * L + base;
  for (int j = threadIdx.x; j < n; j += blockDim.x) x[bitrev(j, r.logM)] = cmul(fr[j], chirp(j, n));
  __syncthreads();
  bluestein_core(x, r, chirp_fft, tw, logMmax);
  const double sc = (normalise ? 1.0 / n : 1.0) / M;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const cplx c = cmul(x[bitrev(q, r.logM)], chirp(q, n));
    H[(base + q) * B + b] = {c.x * sc, c.y * sc};
  }
}

// Synthesis of ring k, map b, with the bins taken either from the
// map-fastest bin array H (scaled by `scale`), or folded from the per-order
// GEMM output Y of the inverse transform:
//   H[q] = sum_{m = q mod n, |m| < L} G'_m(theta_k),
//   G'_m(theta_k) = Y[slot(m)][k][col(m, b)] (complex, two doubles).
// Spin 0: slot(m) = |m|, col = (m < 0 ? 2B : 0) + 2b;  spin != 0:
// slot(m) = m + L - 1, col = 2b.  Summation order over m is fixed
// (ascending m), so results are deterministic.
__global__ __launch_bounds__(256) void ring_synthesis_kernel(const RingDesc* __restrict__ rings,
                                                             const cplx* __restrict__ chirp_fft,
                                                             const cplx* __restrict__ tw, int logMmax, int L,
                                                             const cplx* __restrict__ H, int scale_inv_n,
                                                             const double* __restrict__ Y, int spin0, int ncols,
                                                             cplx* __restrict__ f, int B) {
  const int k = blockIdx.x, b = blockIdx.y;
  const RingDesc r = rings[k];
  const int M = 1 << r.logM, n = r.n;
  const int64_t base = (int64_t)k * k;
  cplx* x = lds_buf;
  for (int i = threadIdx.x; i < M; i += blockDim.x) x[i] = {0.0, 0.0};
  __syncthreads();
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    cplx h = {0.0, 0.0};
    if (Y == nullptr) {
      h = H[(base + q) * B + b];
      if (scale_inv_n) { h.x /= n; h.y /= n; }
    } else {
      // orders m in (-L, L) with m = q (mod n), q taken in [0, n)
      int mstart = q - ((q + L - 1) / n) * n;  // smallest m >= -(L-1) congruent to q
      for (int m = mstart; m <= L - 1; m += n) {
        int slot, col;
        if (spin0) { slot = m < 0 ? -m : m; col = (m < 0 ? 2 * B : 0) + 2 * b; }
        else { slot = m + L - 1; col = 2 * b; }
        const double* y = Y + ((int64_t)slot * L + k) * ncols + col;
        h.x += y[0];
        h.y += y[1];
      }
    }
    x[bitrev(q, r.logM)] = cmul(cconj(h), chirp(q, n));
  }
  __syncthreads();
  bluestein_core(x, r, chirp_fft, tw, logMmax);
  const double sc = 1.0 / M;
  cplx* fr = f + (int64_t)b * L * L + base;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const cplx c = cmul(x[bitrev(j, r.logM)], chirp(j, n));
    fr[j] = {c.x * sc, -c.y * sc};
  }
}

__global__ void twiddle_kernel(cplx* tw, int Mmax) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < Mmax / 2) {
    double s, c;
    sincospi(-2.0 * (double)j / (double)Mmax, &s, &c);
    tw[j] = {c, s};
  }
}

void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 65536) OSHT_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

}  // namespace

void build_chirps(Plan& p) {
  const int L = p.L;
  std::vector<RingDesc> rings(L);
  int64_t off = 0;
  int maxlog = 0;
  for (int k = 0; k < L; ++k) {
    const int n = 2 * k + 1;
    int logM = 0;
    while ((1 << logM) < 2 * n - 1) ++logM;
    rings[k] = RingDesc{n, logM, off};
    off += (int64_t)1 << logM;
    maxlog = std::max(maxlog, logM);
  }
  p.max_logM = std::max(maxlog, 1);
  upload(p.d_rings, rings);
  const int Mmax = 1 << p.max_logM;
  p.d_twiddle.alloc(sizeof(cplx) * (Mmax / 2));
  hipLaunchKernelGGL(twiddle_kernel, dim3(ceil_div(Mmax / 2, 256)), dim3(256), 0, 0, p.d_twiddle.as<cplx>(), Mmax);
  OSHT_HIP(hipGetLastError());
  p.d_chirp.alloc(sizeof(cplx) * off);
  const size_t lds = sizeof(cplx) * (size_t)Mmax;
  allow_lds((const void*)chirp_kernel, lds);
  hipLaunchKernelGGL(chirp_kernel, dim3(L), dim3(256), lds, 0, p.d_rings.as<RingDesc>(), p.d_chirp.as<cplx>(),
                     p.d_twiddle.as<cplx>(), p.max_logM);
  OSHT_HIP(hipGetLastError());
}

void launch_ring_analysis(const Plan& p, const double* f, double* H, int64_t B, bool normalise, hipStream_t st) {
  const size_t lds = sizeof(cplx) * ((size_t)1 << p.max_logM);
  allow_lds((const void*)ring_analysis_kernel, lds);
  hipLaunchKernelGGL(ring_analysis_kernel, dim3(p.L, (unsigned)B), dim3(256), lds, st, p.d_rings.as<RingDesc>(),
                     p.d_chirp.as<cplx>(), p.d_twiddle.as<cplx>(), p.max_logM, p.L,
                     reinterpret_cast<const cplx*>(f), reinterpret_cast<cplx*>(H), (int)B, normalise ? 1 : 0);
  OSHT_HIP(hipGetLastError());
}

void launch_ring_synthesis(const Plan& p, const double* H, int scale_inv_n, const double* Y, double* f, int64_t B,
                           hipStream_t st) {
  const size_t lds = sizeof(cplx) * ((size_t)1 << p.max_logM);
  allow_lds((const void*)ring_synthesis_kernel, lds);
  hipLaunchKernelGGL(ring_synthesis_kernel, dim3(p.L, (unsigned)B), dim3(256), lds, st, p.d_rings.as<RingDesc>(),
                     p.d_chirp.as<cplx>(), p.d_twiddle.as<cplx>(), p.max_logM, p.L,
                     reinterpret_cast<const cplx*>(H), scale_inv_n, Y, p.spin == 0 ? 1 : 0,
                     p.ncols_per_map * (int)B, reinterpret_cast<cplx*>(f), (int)B);
  OSHT_HIP(hipGetLastError());
}

}  // namespace osht
