// Blocked forward sweep (Procedure 1 with the order loop taken b levels at
// a time).
//
// Procedure 1 removes, before order m is solved, the aliases of every order
// |m'| > |m| from the rings k >= |m| (Eq. signal_update).  In the Fourier
// domain ring k receives order m' in bin (m' mod n_k), n_k = 2k+1, and
// g_m[k] = H_k[m mod n_k] - sum_{m' = m (mod n_k), |m'| > k} G'_{m'}(theta_k).
// An alias m' = m + j n_k (j != 0) has |m'| >= 2k+1-|m|, so within a block of
// levels [q0, q1) only the rows k < (q1+|m|-1)/2 of an order receive aliases
// from other orders of the same block.  For block [q0, q1):
//   1. gather   h_m[k] = H_k[m mod n_k] - sum over solved orders (|m'| >= q1)
//   2. GEMM     Y_m = Q_m h_m     (Q_m = [P_m^{-1}; A_m^top P_m^{-1}])
//   3. solve    for the unknown alias rows u = (m, k) of the block:
//                 delta_u = beta_u - sum_{u'} W_{u,u'} delta_{u'},
//               beta_u = sum_{m'} (Y_{m'})[K(m') + k]   (= C_{m'} h_{m'} at ring k),
//               W_{u,u'} = Q_{m'}[K(m') + k, k' - |m'|] for u' = (m', k');
//               a triangular system solved level by level (descending |m|),
//   4. correct  Y_m -= Q_m[:, 0:q1-|m|] delta_m   (so Y_m = Q_m (h_m - delta_m)).
// Afterwards Y_m holds f_m and the exact aliases G'_m on the rings k < |m|,
// which later blocks read in step 1.  All sums run in a fixed order.

#include <unistd.h>

#include <algorithm>
#include <cstdio>
#include <string>
#include <cstdlib>

#include "xform.hpp"

namespace osht {
void launch_ring_synthesis(const Plan& p, const double* H, int scale_inv_n, double* f, int64_t B, hipStream_t st,
                           int64_t real_maps = 0);
}

namespace osht {

namespace {

// One thread per (row r, complex column cc = sgn * B + b): both doubles of
// the complex RHS entry, with the alias search shared by re and im.
// ring_cut: orders |m'| >= ring_cut[k] have every Legendre value on ring k
// below 2^-80, so their alias values there are below FP64 resolution of the
// bin and are not subtracted.
__global__ __launch_bounds__(256) void block_gather_kernel(Geo g, const Slot* __restrict__ slots,
                                                           const int32_t* __restrict__ slot_list, int q1, int kthr,
                                                           const int32_t* __restrict__ ring_cut,
                                                           const double2* __restrict__ H, const double* __restrict__ Y,
                                                           double2* __restrict__ X) {
  const int slot = slot_list[blockIdx.y];
  const Slot sl = slots[slot];
  const int nc = g.ncols >> 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = e / nc, cc = e - r * nc;
  if (r >= sl.R) return;
  const int sgn = (g.s == 0) ? cc / g.B : 0;
  const int b = cc - sgn * g.B;
  const int m = sgn ? -sl.m : sl.m;
  const int am = m < 0 ? -m : m;
  const int k = am + r, n = 2 * k + 1;
  if (k < kthr) return;  // many aliases: wide_gather_kernel
  const int bin = pmod(m, n);
  double2 v = H[((int64_t)k * k + bin) * g.B + b];
  const int cut = ring_cut[k];
  const int start = bin - ((bin + g.L - 1) / n) * n;
  // only orders solved in earlier blocks (|m'| >= q1); four loads in flight,
  // an excluded entry loading Y[0] and subtracting nothing, so the
  // subtractions keep ascending m' order
  int mp = start;
  for (; mp + 3 * n <= g.L - 1; mp += 4 * n) {
    double2 a[4];
    bool use[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int q = mp + t * n, aq = q < 0 ? -q : q;
      use[t] = q != m && aq >= q1 && aq < cut;
      a[t] = *reinterpret_cast<const double2*>(Y + (use[t] ? alias_index(g, slots, q, k, b, 0) : 0));
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (use[t]) {
        v.x -= a[t].x;
        v.y -= a[t].y;
      }
    }
  }
  for (; mp <= g.L - 1; mp += n) {
    const int amp = mp < 0 ? -mp : mp;
    if (mp == m || amp < q1 || amp >= cut) continue;
    const double2 a = *reinterpret_cast<const double2*>(Y + alias_index(g, slots, mp, k, b, 0));
    v.x -= a.x;
    v.y -= a.y;
  }
  X[((int64_t)slot * g.L + r) * nc + cc] = v;
}

// The rows of small rings (k < kthr) alias up to ~(2L-1)/n_k solved orders.
// One workgroup of 1024 threads per (slot, row): threads split the columns
// and, for each column, the alias list into C interleaved chunks whose
// partial sums are reduced in a fixed order through LDS.  Each thread keeps
// four alias loads in flight (an excluded order loads Y[0] instead and is
// dropped by a select).
constexpr int kWideThreads = 1024;
// Rings with more aliased orders per bin than this go to the wide kernel: a
// block-gather thread then walks at most 8 batches of four alias loads
// (32 and 16 measured equal, 64 slower by 0.6 us per block at L = 1024).
constexpr int kWideAliases = 32;
__global__ __launch_bounds__(kWideThreads) void wide_gather_kernel(Geo g, const Slot* __restrict__ slots,
                                                                   const int32_t* __restrict__ wide_slot,
                                                                   const int32_t* __restrict__ wide_row, int q1,
                                                                   const int32_t* __restrict__ ring_cut,
                                                                   const double2* __restrict__ H,
                                                                   const double* __restrict__ Y,
                                                                   double2* __restrict__ X) {
  __shared__ double2 part[kWideThreads];
  const int slot = wide_slot[blockIdx.x], r = wide_row[blockIdx.x];
  const Slot sl = slots[slot];
  const int nc = g.ncols >> 1;
  const int cw = nc < kWideThreads ? nc : kWideThreads;  // columns in flight
  const int C = kWideThreads / cw;                        // alias chunks per column
  const int ci = threadIdx.x % cw, chunk = threadIdx.x / cw;
  for (int cc0 = 0; cc0 < nc; cc0 += cw) {
    const int cc = cc0 + ci;
    double2 acc = {0.0, 0.0};
    int bin = 0, m = 0, k = 0, b = 0;
    if (chunk < C && cc < nc) {
      const int sgn = (g.s == 0) ? cc / g.B : 0;
      b = cc - sgn * g.B;
      m = sgn ? -sl.m : sl.m;
      k = (m < 0 ? -m : m) + r;
      const int n = 2 * k + 1;
      bin = pmod(m, n);
      const int cut = ring_cut[k];  // as in block_gather_kernel
      const int start = bin - ((bin + g.L - 1) / n) * n;
      const int step = C * n;
      int mp = start + chunk * n;
      for (; mp + 3 * step <= g.L - 1; mp += 4 * step) {
        double2 a[4];
        bool use[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int q = mp + t * step, aq = q < 0 ? -q : q;
          use[t] = q != m && aq >= q1 && aq < cut;  // then |q| > k and the alias row exists
          a[t] = *reinterpret_cast<const double2*>(Y + (use[t] ? alias_index(g, slots, q, k, b, 0) : 0));
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          acc.x += use[t] ? a[t].x : 0.0;
          acc.y += use[t] ? a[t].y : 0.0;
        }
      }
      for (; mp <= g.L - 1; mp += step) {
        const int amp = mp < 0 ? -mp : mp;
        if (mp == m || amp < q1 || amp >= cut) continue;
        const double2 a = *reinterpret_cast<const double2*>(Y + alias_index(g, slots, mp, k, b, 0));
        acc.x += a.x;
        acc.y += a.y;
      }
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (chunk == 0 && cc < nc) {
      double2 v = H[((int64_t)k * k + bin) * g.B + b];
      for (int c = 0; c < C; ++c) {
        v.x -= part[c * cw + ci].x;
        v.y -= part[c * cw + ci].y;
      }
      X[((int64_t)slot * g.L + r) * nc + cc] = v;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int order_col(const Geo& g, int m, int j) {
  return (g.s == 0 && m < 0) ? 2 * g.B + j : j;
}

// Alias unknowns of one block, solved level by level (descending |m|):
//   delta_u = beta_u - sum_{u'} W_{u,u'} delta_{u'},
//   beta_u  = sum over the alias sources m' of u = (m, k) of (Y_{m'})[K(m') + k].
// The block's W (values and block-local columns) sits in LDS together with
// delta for `cpw` columns; workgroup g handles columns [g*cpw, (g+1)*cpw) of
// the 2B map-part columns.  Writes delta into D[slot][r][col].
__global__ __launch_bounds__(512) void delta_solve_kernel(Geo g, int u0, int nu, int nlev, int cpw,
                                                          const int32_t* __restrict__ lev_ptr,
                                                          const int32_t* __restrict__ unk_slot,
                                                          const int32_t* __restrict__ unk_r,
                                                          const int32_t* __restrict__ unk_m,
                                                          const int32_t* __restrict__ src_ptr,
                                                          const int32_t* __restrict__ src_slot,
                                                          const int32_t* __restrict__ src_row,
                                                          const int32_t* __restrict__ src_m,
                                                          const int64_t* __restrict__ w_ptr,
                                                          const int32_t* __restrict__ w_col,
                                                          const double* __restrict__ w_val, const double* __restrict__ Y,
                                                          double* __restrict__ D, int bD) {
  extern __shared__ double lds[];
  const int64_t wbase = w_ptr[u0];
  const int nw = (int)(w_ptr[u0 + nu] - wbase);
  double* dl = lds;                                   // nu * cpw
  double* wv = lds + (size_t)nu * cpw;                // nw
  int32_t* wc = reinterpret_cast<int32_t*>(wv + nw);  // nw
  int32_t* wp = wc + nw;                              // nu + 1 (block-relative row starts)
  const int j0 = blockIdx.x * cpw;
  const int J = 2 * g.B;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) {
    wv[i] = w_val[wbase + i];
    wc[i] = w_col[wbase + i];
  }
  for (int i = threadIdx.x; i <= nu; i += blockDim.x) wp[i] = (int32_t)(w_ptr[u0 + i] - wbase);
  // beta for every unknown and column of this group
  for (int e = threadIdx.x; e < nu * cpw; e += blockDim.x) {
    const int ul = e / cpw, jj = e - ul * cpw, j = j0 + jj;
    double acc = 0.0;
    if (j < J) {
      const int u = u0 + ul;
      for (int s = src_ptr[u]; s < src_ptr[u + 1]; ++s)
        acc += Y[((int64_t)src_slot[s] * g.L + src_row[s]) * g.ncols + order_col(g, src_m[s], j)];
    }
    dl[e] = acc;
  }
  __syncthreads();
  // level-ordered substitution, LDS only; each (unknown, column) item is
  // reduced by a group of G lanes (strided partial sums, then a fixed
  // butterfly over the group), so the per-level critical path is
  // ~len(W row)/G steps
  constexpr int G = 8;
  const int grp = threadIdx.x / G, lg = threadIdx.x % G, ngrp = blockDim.x / G;
  for (int lv = 0; lv < nlev; ++lv) {
    const int a = lev_ptr[lv] - u0, b = lev_ptr[lv + 1] - u0;
    const int items = (b - a) * cpw;
    for (int e0 = 0; e0 < items; e0 += ngrp) {
      const int e = e0 + grp;
      double part = 0.0;
      int ul = 0, jj = 0;
      if (e < items) {
        ul = a + e / cpw;
        jj = e % cpw;
        int w = wp[ul] + lg;
        const int we = wp[ul + 1];
        // four W entries per lane in flight before their delta reads
        for (; w + 3 * G < we; w += 4 * G) {
          const double v0 = wv[w], v1 = wv[w + G], v2 = wv[w + 2 * G], v3 = wv[w + 3 * G];
          const int c0 = wc[w], c1 = wc[w + G], c2 = wc[w + 2 * G], c3 = wc[w + 3 * G];
          part += v0 * dl[c0 * cpw + jj];
          part += v1 * dl[c1 * cpw + jj];
          part += v2 * dl[c2 * cpw + jj];
          part += v3 * dl[c3 * cpw + jj];
        }
        for (; w < we; w += G) part += wv[w] * dl[wc[w] * cpw + jj];
      }
#pragma unroll
      for (int off = 1; off < G; off <<= 1) part += __shfl_xor(part, off, G);
      if (e < items && lg == 0) dl[ul * cpw + jj] -= part;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nu * cpw; e += blockDim.x) {
    const int ul = e / cpw, jj = e - ul * cpw, j = j0 + jj;
    if (j < J) {
      const int u = u0 + ul;
      D[((int64_t)unk_slot[u] * bD + unk_r[u]) * g.ncols + order_col(g, unk_m[u], j)] = dl[e];
    }
  }
}

// The same unknowns through the block's precomputed inverse:
// delta = (I + W)^{-1} beta, beta_u the sum of the alias values of u's
// sources.  With the inverse's column u repeated for every source of u
// (Minv_s, one column per source, sources ordered by their unknown),
// delta = Minv_s s, s the vector of the sources' alias values: one FP64
// matrix-core product that reads the alias rows of Y directly.
//
// Rows are unknowns, k runs over the block's sources s (global index s0 + k):
// A[r][k] = Minv_s[k * ld + r] (column-major, lower triangular in the
// unknown order), B[k][j] = Y[row(s) * ncols + order_col(m_s, j)] with
// src_yrow[s] = 2 row(s) + (m_s < 0 on spin 0).  Workgroup (x, y) computes
// unknowns [16x, 16x + 16) and columns [32y, 32y + 32) of the 2B map-part
// columns; its waves split the sources [0, src_ptr[u0 + 16x + 16] - s0) (the
// triangle) into equal chunks, and the partial tiles are summed in LDS in
// wave order.  Writes delta into D[slot][r][col].
constexpr int kDeltaWaves = 16;
// Workgroups per 16-row tile, each over one part of the sources (1 or 2):
// the kernel is bound by its chain of dependent loads, so halving each
// wave's share of the sources shortens it.
constexpr int kDeltaSplit = 2;
__global__ __launch_bounds__(64 * kDeltaWaves) void delta_apply_kernel(
    Geo g, int u0, int nu, int s0, const int32_t* __restrict__ src_ptr, const int32_t* __restrict__ src_yrow,
    const double* __restrict__ Minv, int ld, const double* __restrict__ Y, const int32_t* __restrict__ unk_slot,
    const int32_t* __restrict__ unk_r, const int32_t* __restrict__ unk_m, double* __restrict__ D, int bD) {
  typedef double dbl4 __attribute__((ext_vector_type(4)));
  __shared__ double red[kDeltaWaves][2][16][16];
  const int J = 2 * g.B;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row0 = blockIdx.x * 16, col0 = blockIdx.y * 32;
  const int kt = src_ptr[u0 + min(nu, row0 + 16)] - s0;
  // with gridDim.z = 2 each workgroup takes one half of the sources and the
  // two partial tiles are added into the zeroed D: two addends onto zero
  // give the same bits in either order
  const int kh = (kt + 1) / 2;
  const int zb = gridDim.z > 1 ? (int)blockIdx.z * kh : 0, ze = gridDim.z > 1 ? min(kt, zb + kh) : kt;
  const int chunk = ((ze - zb + kDeltaWaves - 1) / kDeltaWaves + 3) & ~3;
  const int kb = zb + wave * chunk, ke = min(ze, kb + chunk);
  const int r = row0 + (lane & 15), q = lane >> 4;
  const int c0 = col0 + (lane & 15), c1 = c0 + 16;
  const bool rok = r < nu, c0ok = c0 < J, c1ok = c1 < J;
  dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  // batches of four k-steps, double-buffered in registers: the data loads of
  // batch i + 1 are in flight while batch i runs on the matrix cores, and the
  // source-row indices they need were loaded one batch earlier still, so no
  // batch waits on two dependent loads; k beyond the wave's range loads zeros
  double a[2][4], b0[2][4], b1[2][4];
  int yiA[4], yiB[4];
  auto load_idx = [&](int* py, int kbase) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = kbase + 4 * t + q;
      py[t] = k < ke ? src_yrow[s0 + k] : 0;
    }
  };
  auto load = [&](double* pa, double* pb0, double* pb1, const int* py, int kbase) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = kbase + 4 * t + q;
      const bool kok = k < ke;
      const int yr = py[t];
      const double* yrow = Y + (int64_t)(yr >> 1) * g.ncols + ((yr & 1) ? J : 0);
      pa[t] = (rok && kok) ? Minv[(int64_t)k * ld + r] : 0.0;
      pb0[t] = (c0ok && kok) ? yrow[c0] : 0.0;
      pb1[t] = (c1ok && kok) ? yrow[c1] : 0.0;
    }
  };
  auto mfma4 = [&](const double* pa, const double* pb0, const double* pb1) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[t], pb0[t], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[t], pb1[t], acc1, 0, 0, 0);
    }
  };
  const int nbat = ke > kb ? (ke - kb + 15) / 16 : 0;
  // at the top of each pair: a[0] holds batch i, yiB the indices of batch i+1
  if (nbat > 0) load_idx(yiA, kb);
  if (nbat > 1) load_idx(yiB, kb + 16);
  if (nbat > 0) load(a[0], b0[0], b1[0], yiA, kb);
  for (int i = 0; i < nbat; i += 2) {
    if (i + 2 < nbat) load_idx(yiA, kb + 16 * (i + 2));
    if (i + 1 < nbat) load(a[1], b0[1], b1[1], yiB, kb + 16 * (i + 1));
    mfma4(a[0], b0[0], b1[0]);
    if (i + 1 < nbat) {
      if (i + 3 < nbat) load_idx(yiB, kb + 16 * (i + 3));
      if (i + 2 < nbat) load(a[0], b0[0], b1[0], yiA, kb + 16 * (i + 2));
      mfma4(a[1], b0[1], b1[1]);
    }
  }
  // accumulator register v of lane l holds row l / 16 + 4 v, column l % 16
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    red[wave][0][q + 4 * v][lane & 15] = acc0[v];
    red[wave][1][q + 4 * v][lane & 15] = acc1[v];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 512; e += 64 * kDeltaWaves) {
    const int ct = e >> 8, i = (e >> 4) & 15, c = e & 15;
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kDeltaWaves; ++w) sum += red[w][ct][i][c];
    const int ul = row0 + i, j = col0 + 16 * ct + c;
    if (ul < nu && j < J) {
      const int u = u0 + ul;
      double* dp = D + ((int64_t)unk_slot[u] * bD + unk_r[u]) * g.ncols + order_col(g, unk_m[u], j);
      if (gridDim.z > 1) unsafeAtomicAdd(dp, sum);
      else *dp = sum;
    }
  }
}

// ---------------------------------------------------------------- adjoint
// The adjoint of the blocked forward runs the blocks in ascending order.
// For block [q0, q1) with y_m = Q_m (h_m - E delta), delta = (I + W)^{-1} A Q h:
//   z = Q^T ybar;  (I + W^T) eps = z restricted to the unknowns;
//   hbar = z - Q^T A^T eps;  Hbar_k[m mod n_k] = hbar_m[k] (m owns that bin).
// ybar_m holds flm_bar on its coefficient rows and, on an alias row k < |m|,
// -Hbar_k[m mod n_k] when the owner of that bin (the order congruent to m in
// [-k, k]) lies below the block; owners inside the block are covered by eps.

// ybar for the block's slots: X[slot][i][col], i < K + |m|.
__global__ __launch_bounds__(256) void fadj_block_gather_kernel(Geo g, const Slot* __restrict__ slots,
                                                                const int32_t* __restrict__ slot_list, int q0,
                                                                const double* __restrict__ flmbar,
                                                                const double* __restrict__ H, double* __restrict__ X) {
  const int slot = slot_list[blockIdx.y];
  const Slot sl = slots[slot];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = e / g.ncols, col = e % g.ncols;
  int sgn, b, part, m;
  decode_col(g, sl, col, sgn, b, part, m);
  const int am = m < 0 ? -m : m;
  if (i >= sl.K + am) return;
  double v = 0.0;
  if (i < sl.K) {
    const int l = sl.l0 + i;
    v = flmbar[((int64_t)b * g.L * g.L + (int64_t)l * l + l + m) * 2 + part];
    if (g.s == 0 && sgn && (am & 1)) v = -v;
  } else {
    const int k = i - sl.K, n = 2 * k + 1;
    const int owner = pmod(m + k, n) - k;  // the order congruent to m in [-k, k]
    if ((owner < 0 ? -owner : owner) < q0) v = -H[(((int64_t)k * k + pmod(m, n)) * g.B + b) * 2 + part];
  }
  X[((int64_t)slot * g.L + i) * g.ncols + col] = v;
}

// Hbar_k[m mod n_k] = Z[slot][k - |m|][col] for the block's slots.
__global__ __launch_bounds__(256) void fadj_block_scatter_kernel(Geo g, const Slot* __restrict__ slots,
                                                                 const int32_t* __restrict__ slot_list,
                                                                 const double* __restrict__ Y, double* __restrict__ H) {
  const int slot = slot_list[blockIdx.y];
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

// (I + W^T) eps = zeta, ascending levels, in LDS; zeta_u = Z of the owner of
// u at its ring.  Then E[source slot][k - q0][col] = eps_u for every alias
// source of u = (m, k) (each (source, k) pair has exactly one owner u).
__global__ __launch_bounds__(512) void eps_solve_kernel(Geo g, int u0, int nu, int nlev, int cpw, int q0,
                                                        const int32_t* __restrict__ lev_ptr,
                                                        const int32_t* __restrict__ unk_slot,
                                                        const int32_t* __restrict__ unk_r,
                                                        const int32_t* __restrict__ unk_m,
                                                        const int32_t* __restrict__ src_ptr,
                                                        const int32_t* __restrict__ src_slot,
                                                        const int32_t* __restrict__ src_m,
                                                        const int64_t* __restrict__ wt_ptr,
                                                        const int32_t* __restrict__ wt_row,
                                                        const double* __restrict__ wt_val, const double* __restrict__ Y,
                                                        double* __restrict__ D, int bD) {
  extern __shared__ double lds[];
  const int64_t wbase = wt_ptr[u0];
  const int nw = (int)(wt_ptr[u0 + nu] - wbase);
  double* el = lds;                                    // nu * cpw
  double* wv = lds + (size_t)nu * cpw;                 // nw
  int32_t* wr = reinterpret_cast<int32_t*>(wv + nw);   // nw
  int32_t* wp = wr + nw;                               // nu + 1
  const int j0 = blockIdx.x * cpw;
  const int J = 2 * g.B;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) {
    wv[i] = wt_val[wbase + i];
    wr[i] = wt_row[wbase + i];
  }
  for (int i = threadIdx.x; i <= nu; i += blockDim.x) wp[i] = (int32_t)(wt_ptr[u0 + i] - wbase);
  for (int e = threadIdx.x; e < nu * cpw; e += blockDim.x) {
    const int ul = e / cpw, jj = e - ul * cpw, j = j0 + jj;
    const int u = u0 + ul;
    el[e] = (j < J) ? Y[((int64_t)unk_slot[u] * g.L + unk_r[u]) * g.ncols + order_col(g, unk_m[u], j)] : 0.0;
  }
  __syncthreads();
  // lev_ptr lists the block's levels in descending |m|; W^T couples each
  // unknown to unknowns of lower levels, so walk the list backwards
  constexpr int G = 8;
  const int grp = threadIdx.x / G, lg = threadIdx.x % G, ngrp = blockDim.x / G;
  for (int lv = nlev - 1; lv >= 0; --lv) {
    const int a = lev_ptr[lv] - u0, b = lev_ptr[lv + 1] - u0;
    const int items = (b - a) * cpw;
    for (int e0 = 0; e0 < items; e0 += ngrp) {
      const int e = e0 + grp;
      double part = 0.0;
      int ul = 0, jj = 0;
      if (e < items) {
        ul = a + e / cpw;
        jj = e % cpw;
        for (int w = wp[ul] + lg; w < wp[ul + 1]; w += G) part += wv[w] * el[wr[w] * cpw + jj];
      }
#pragma unroll
      for (int off = 1; off < G; off <<= 1) part += __shfl_xor(part, off, G);
      if (e < items && lg == 0) el[ul * cpw + jj] -= part;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nu * cpw; e += blockDim.x) {
    const int ul = e / cpw, jj = e - ul * cpw, j = j0 + jj;
    if (j >= J) continue;
    const int u = u0 + ul;
    const int am = unk_m[u] < 0 ? -unk_m[u] : unk_m[u];
    const int k = unk_r[u] + am;
    for (int s = src_ptr[u]; s < src_ptr[u + 1]; ++s)
      D[((int64_t)src_slot[s] * bD + (k - q0)) * g.ncols + order_col(g, src_m[s], j)] = el[e];
  }
}

__global__ void fill_zero_kernel(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void gather_values_kernel(const double* __restrict__ src, const int64_t* __restrict__ idx,
                                     double* __restrict__ dst, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

template <class T>
void put_vec(DevBuf& d, const std::vector<T>& h) {
  d.alloc(std::max<size_t>(h.size(), 1) * sizeof(T));
  if (!h.empty()) OSHT_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

}  // namespace

namespace {

// (I + W)^{-1} of every block, by rows: with M = (I + W)^{-1}, M = I - W M,
// and W only couples an unknown to unknowns of earlier (higher) levels, so
// row u of M is e_u minus the W-weighted rows of M already computed.  The
// product runs in FP64 on the host, once per block structure; M is lower
// triangular and is stored column-major for the device product.
void build_delta_inverses(Plan& p) {
  FwdBlocks& fb = p.fb;
  const int nblk = (int)fb.q0.size();
  if (!fb.dense) {
    fb.minv_off.clear();
    fb.minv_ld.clear();
    fb.d_minv.release();
    return;
  }
  fb.minv_off.assign(nblk + 1, 0);
  fb.minv_ld.assign(nblk, 0);
  int64_t tot = 0;
  for (int blk = 0; blk < nblk; ++blk) {
    const int u0 = fb.unk_ptr[blk], nu = fb.unk_ptr[blk + 1] - u0;
    const int ns = fb.src_ptr[u0 + nu] - fb.src_ptr[u0];
    fb.minv_ld[blk] = (int32_t)round_up(std::max(nu, 1), 16);
    fb.minv_off[blk] = tot;
    tot += (int64_t)fb.minv_ld[blk] * ns;
  }
  fb.minv_off[nblk] = tot;
  fb.d_minv.alloc(sizeof(double) * (size_t)std::max<int64_t>(tot, 1));
  const int64_t nw = fb.w_ptr.back();
  std::vector<double> wv((size_t)nw);
  if (nw > 0) OSHT_HIP(hipMemcpy(wv.data(), fb.d_w_val.p, sizeof(double) * nw, hipMemcpyDeviceToHost));
  std::vector<double> Mr, Mt;
  for (int blk = 0; blk < nblk; ++blk) {
    const int u0 = fb.unk_ptr[blk], nu = fb.unk_ptr[blk + 1] - u0, ld = fb.minv_ld[blk];
    if (nu == 0) continue;
    Mr.assign((size_t)nu * nu, 0.0);
    for (int ul = 0; ul < nu; ++ul) {
      double* row = &Mr[(size_t)ul * nu];
      row[ul] = 1.0;
      for (int64_t w = fb.w_ptr[u0 + ul]; w < fb.w_ptr[u0 + ul + 1]; ++w) {
        const int c = fb.w_col[w];
        OSHT_CHECK(c < ul, OSHT_ENOTSUP, "alias system not ordered by level");
        const double x = wv[(size_t)w];
        const double* rc = &Mr[(size_t)c * nu];
        for (int q = 0; q <= c; ++q) row[q] -= x * rc[q];
      }
    }
    // column s (a source of unknown c) holds column c of M: rows ul >= c
    const int sb = fb.src_ptr[u0], ns = fb.src_ptr[u0 + nu] - sb;
    Mt.assign((size_t)ld * ns, 0.0);
    for (int c = 0; c < nu; ++c)
      for (int sg = fb.src_ptr[u0 + c]; sg < fb.src_ptr[u0 + c + 1]; ++sg)
        for (int ul = c; ul < nu; ++ul) Mt[(size_t)(sg - sb) * ld + ul] = Mr[(size_t)ul * nu + c];
    OSHT_HIP(hipMemcpy(fb.d_minv.as<double>() + fb.minv_off[blk], Mt.data(), sizeof(double) * Mt.size(),
                       hipMemcpyHostToDevice));
  }
  // per source: 2 (slot L + alias row) + (order < 0 on spin 0)
  std::vector<int32_t> yrow(fb.src_slot.size());
  for (size_t i = 0; i < yrow.size(); ++i) {
    const int64_t row = (int64_t)fb.src_slot[i] * p.L + fb.src_row[i];
    OSHT_CHECK(row < (int64_t)1 << 30, OSHT_ENOTSUP, "alias row index out of range");
    yrow[i] = (int32_t)(2 * row + ((p.spin == 0 && fb.src_m[i] < 0) ? 1 : 0));
  }
  put_vec(fb.d_src_yrow, yrow);
}

}  // namespace

void build_fwd_blocks(Plan& p, int b) {
  FwdBlocks& fb = p.fb;
  fb.clear_host();
  fb.b = std::max(1, std::min(b, p.L));
  const int L = p.L, s = p.spin;
  auto slot_of = [&](int m) { return s == 0 ? std::abs(m) : m + L - 1; };
  auto Kof = [&](int m) { return L - std::max(std::abs(m), std::abs(s)); };
  fb.slot_ptr.push_back(0);
  fb.unk_ptr.push_back(0);
  fb.lev_blk_ptr.push_back(0);
  fb.src_ptr.push_back(0);
  fb.w_ptr.push_back(0);
  fb.wt_ptr.push_back(0);
  fb.wide_ptr.push_back(0);
  // rings with more than ~kWideAliases aliased orders per bin:
  // n_k * kWideAliases < 2L - 1
  fb.kthr = 0;
  while ((2 * fb.kthr + 1) * kWideAliases < 2 * L - 1) ++fb.kthr;
  for (int q1 = L; q1 > 0; q1 -= fb.b) {
    const int q0 = std::max(0, q1 - fb.b);
    fb.q0.push_back(q0);
    fb.q1.push_back(q1);
    // slots of the block (descending level)
    for (int am = q1 - 1; am >= q0; --am) {
      fb.slot_list.push_back(slot_of(am));
      if (s != 0 && am > 0) fb.slot_list.push_back(slot_of(-am));
    }
    fb.slot_ptr.push_back((int32_t)fb.slot_list.size());
    // unknowns, level by level; map (m, k) -> block-local index
    const int u0 = (int)fb.unk_m.size();
    std::vector<std::vector<int>> local_of(2 * L);  // index by m + L - 1, vector over k - |m|
    struct Unk { int m, k; std::vector<int> src; };
    std::vector<Unk> unks;
    for (int am = q1 - 1; am >= q0; --am) {
      fb.lev_ptr.push_back(u0 + (int)unks.size());
      for (int m : {am, -am}) {
        if (am == 0 && m != 0) continue;
        for (int k = am; k < q1; ++k) {
          const int n = 2 * k + 1;
          std::vector<int> src;
          const int bin = ((m % n) + n) % n;
          const int start = bin - ((bin + L - 1) / n) * n;
          for (int mp = start; mp <= L - 1; mp += n) {
            const int amp = std::abs(mp);
            if (mp == m || amp >= q1 || amp < q0 || amp <= k) continue;
            src.push_back(mp);
          }
          if (src.empty()) continue;
          std::vector<int>& lo = local_of[m + L - 1];
          if (lo.empty()) lo.assign(q1 - am, -1);
          lo[k - am] = (int)unks.size();
          unks.push_back(Unk{m, k, src});
        }
        if (am == 0) break;
      }
    }
    fb.lev_ptr.push_back(u0 + (int)unks.size());
    fb.lev_blk_ptr.push_back((int32_t)fb.lev_ptr.size());
    for (const Unk& u : unks) {
      fb.unk_m.push_back(u.m);
      fb.unk_slot.push_back(slot_of(u.m));
      fb.unk_r.push_back(u.k - std::abs(u.m));
      for (int mp : u.src) {
        const int sp = slot_of(mp);
        fb.src_slot.push_back(sp);
        fb.src_row.push_back(Kof(mp) + u.k);
        fb.src_m.push_back(mp);
        // W row: alias row (K(m') + k) of Q_{m'} at the columns of m''s own unknowns
        const std::vector<int>& lo = local_of[mp + L - 1];
        const Slot& sl = p.slots[sp];
        for (size_t c = 0; c < lo.size(); ++c) {
          if (lo[c] < 0) continue;
          fb.w_col.push_back(lo[c]);
          fb.w_idx.push_back(sl.offQ + (int64_t)c * sl.ldQ + (Kof(mp) + u.k));
        }
      }
      fb.src_ptr.push_back((int32_t)fb.src_slot.size());
      fb.w_ptr.push_back((int64_t)fb.w_col.size());
    }
    fb.unk_ptr.push_back((int32_t)fb.unk_m.size());
    fb.max_unk = std::max(fb.max_unk, (int)unks.size());
    // W^T for the forward adjoint: column u' of W as a list of (u, value),
    // u in the order of the rows of W
    {
      const int nu = (int)unks.size();
      std::vector<std::vector<std::pair<int32_t, int64_t>>> col(nu);
      const int64_t wb = fb.w_ptr[u0];
      for (int ul = 0; ul < nu; ++ul)
        for (int64_t w = fb.w_ptr[u0 + ul]; w < fb.w_ptr[u0 + ul + 1]; ++w)
          col[fb.w_col[w]].push_back({ul, fb.w_idx[w]});
      (void)wb;
      for (int c = 0; c < nu; ++c) {
        for (const auto& e : col[c]) {
          fb.wt_row.push_back(e.first);
          fb.wt_idx.push_back(e.second);
        }
        fb.wt_ptr.push_back((int64_t)fb.wt_row.size());
      }
    }
    // rows of small rings gathered by the wide kernel
    for (int i = fb.slot_ptr[fb.slot_ptr.size() - 2]; i < fb.slot_ptr.back(); ++i) {
      const int sp = fb.slot_list[i];
      const int am = std::abs(p.slots[sp].m);
      for (int k = am; k < std::min(fb.kthr, L); ++k) {
        fb.wide_slot.push_back(sp);
        fb.wide_row.push_back(k - am);
      }
    }
    fb.wide_ptr.push_back((int32_t)fb.wide_slot.size());
  }
  put_vec(fb.d_slot_list, fb.slot_list);
  put_vec(fb.d_lev_ptr, fb.lev_ptr);
  put_vec(fb.d_unk_slot, fb.unk_slot);
  put_vec(fb.d_unk_r, fb.unk_r);
  put_vec(fb.d_unk_m, fb.unk_m);
  put_vec(fb.d_src_ptr, fb.src_ptr);
  put_vec(fb.d_src_slot, fb.src_slot);
  put_vec(fb.d_src_row, fb.src_row);
  put_vec(fb.d_src_m, fb.src_m);
  put_vec(fb.d_w_ptr, fb.w_ptr);
  put_vec(fb.d_w_col, fb.w_col);
  put_vec(fb.d_wide_slot, fb.wide_slot);
  put_vec(fb.d_wide_row, fb.wide_row);
  put_vec(fb.d_wt_ptr, fb.wt_ptr);
  put_vec(fb.d_wt_row, fb.wt_row);
  const int64_t nw = (int64_t)fb.w_idx.size();
  fb.d_w_val.alloc(std::max<int64_t>(nw, 1) * sizeof(double));
  if (nw > 0) {
    DevBuf d_idx;
    put_vec(d_idx, fb.w_idx);
    hipLaunchKernelGGL(gather_values_kernel, dim3((unsigned)ceil_div(nw, 256)), dim3(256), 0, 0,
                       p.d_Q.as<double>(), d_idx.as<int64_t>(), fb.d_w_val.as<double>(), nw);
    OSHT_HIP(hipGetLastError());
    OSHT_HIP(hipDeviceSynchronize());
  }
  fb.w_idx.clear();
  fb.w_idx.shrink_to_fit();
  build_delta_inverses(p);
  const int64_t nwt = (int64_t)fb.wt_idx.size();
  fb.d_wt_val.alloc(std::max<int64_t>(nwt, 1) * sizeof(double));
  if (nwt > 0) {
    DevBuf d_idx;
    put_vec(d_idx, fb.wt_idx);
    hipLaunchKernelGGL(gather_values_kernel, dim3((unsigned)ceil_div(nwt, 256)), dim3(256), 0, 0,
                       p.d_Q.as<double>(), d_idx.as<int64_t>(), fb.d_wt_val.as<double>(), nwt);
    OSHT_HIP(hipGetLastError());
    OSHT_HIP(hipDeviceSynchronize());
  }
  fb.wt_idx.clear();
  fb.wt_idx.shrink_to_fit();
  // LDS need of the delta solve per block: delta for cpw columns + W
  fb.max_w = 0;
  for (size_t blk = 0; blk + 1 < fb.unk_ptr.size(); ++blk) {
    const int64_t nw = fb.w_ptr[fb.unk_ptr[blk + 1]] - fb.w_ptr[fb.unk_ptr[blk]];
    fb.max_w = std::max<int64_t>(fb.max_w, nw);
  }
}

void run_forward_blocked(Plan& p, const double* f, double* flm, int64_t B, hipStream_t st, int64_t real_maps) {
  ensure_workspace(p, B);
  const Geo g = geo(p, B);
  const FwdBlocks& fb = p.fb;
  {
    ProfScope ps(p.prof, "ring_analysis", st);
    launch_ring_analysis(p, f, p.w_H.as<double>(), B, true, st, real_maps);
  }
  const int bD = std::max(fb.b, 1);
  const int64_t nD = (int64_t)p.nslots * bD * g.ncols;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(nD, 256), 4096)), dim3(256), 0, st,
                     p.w_D.as<double>(), nD);
  OSHT_HIP(hipGetLastError());
  OSHT_HIP(hipFuncSetAttribute((const void*)delta_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                fb.lds_limit));
  const int nblk = (int)fb.q0.size();
  const GemmTask* bt = p.tab->d_btask.as<GemmTask>();
  for (int blk = 0; blk < nblk; ++blk) {
    const int ns = fb.slot_ptr[blk + 1] - fb.slot_ptr[blk];
    {
      ProfScope ps(p.prof, "gather_forward", st);
      hipLaunchKernelGGL(block_gather_kernel, dim3((unsigned)ceil_div((int64_t)p.L * (g.ncols / 2), 256), ns), dim3(256),
                         0, st, g, p.d_slots.as<Slot>(), fb.d_slot_list.as<int32_t>() + fb.slot_ptr[blk], fb.q1[blk],
                         fb.kthr, p.d_ring_cut.as<int32_t>(), reinterpret_cast<const double2*>(p.w_H.as<double>()),
                         p.w_Y.as<double>(),
                         reinterpret_cast<double2*>(p.w_X.as<double>()));
      OSHT_HIP(hipGetLastError());
      const int nwide = fb.wide_ptr[blk + 1] - fb.wide_ptr[blk];
      if (nwide > 0) {
        hipLaunchKernelGGL(wide_gather_kernel, dim3((unsigned)nwide), dim3(kWideThreads), 0, st, g, p.d_slots.as<Slot>(),
                           fb.d_wide_slot.as<int32_t>() + fb.wide_ptr[blk], fb.d_wide_row.as<int32_t>() + fb.wide_ptr[blk],
                           fb.q1[blk], p.d_ring_cut.as<int32_t>(), reinterpret_cast<const double2*>(p.w_H.as<double>()),
                           p.w_Y.as<double>(), reinterpret_cast<double2*>(p.w_X.as<double>()));
        OSHT_HIP(hipGetLastError());
      }
    }
    const int* tp = &p.tab->h_btask_ptr[2 * blk];
    gemm_tasks_launch(p, bt + tp[0], tp[1] - tp[0], GemmRole::ApplyForward, "apply_forward", st);
    const int u0 = fb.unk_ptr[blk], nu = fb.unk_ptr[blk + 1] - u0;
    if (nu > 0) {
      const int lv0 = fb.lev_blk_ptr[blk], lv1 = fb.lev_blk_ptr[blk + 1];
      const int64_t nw = fb.w_ptr[u0 + nu] - fb.w_ptr[u0];
      const int cpw = fb.cpw;
      const size_t lds = sizeof(double) * ((size_t)nu * cpw + nw) + sizeof(int32_t) * (nw + nu + 1);
      if (fb.dense) {
        ProfScope ps(p.prof, "delta_solve", st);
        const int J = 2 * (int)B;
        hipLaunchKernelGGL(delta_apply_kernel, dim3((unsigned)ceil_div(nu, 16), (unsigned)ceil_div(J, 32), kDeltaSplit),
                           dim3(64 * kDeltaWaves), 0, st, g, u0, nu, fb.src_ptr[u0], fb.d_src_ptr.as<int32_t>(),
                           fb.d_src_yrow.as<int32_t>(), fb.d_minv.as<double>() + fb.minv_off[blk], fb.minv_ld[blk],
                           p.w_Y.as<double>(), fb.d_unk_slot.as<int32_t>(), fb.d_unk_r.as<int32_t>(),
                           fb.d_unk_m.as<int32_t>(), p.w_D.as<double>(), bD);
        OSHT_HIP(hipGetLastError());
      } else {
        ProfScope ps(p.prof, "delta_solve", st);
        hipLaunchKernelGGL(delta_solve_kernel, dim3((unsigned)ceil_div(2 * B, cpw)), dim3(512), lds, st, g, u0, nu,
                           lv1 - lv0 - 1, cpw, fb.d_lev_ptr.as<int32_t>() + lv0, fb.d_unk_slot.as<int32_t>(),
                           fb.d_unk_r.as<int32_t>(), fb.d_unk_m.as<int32_t>(), fb.d_src_ptr.as<int32_t>(),
                           fb.d_src_slot.as<int32_t>(), fb.d_src_row.as<int32_t>(), fb.d_src_m.as<int32_t>(),
                           fb.d_w_ptr.as<int64_t>(), fb.d_w_col.as<int32_t>(), fb.d_w_val.as<double>(),
                           p.w_Y.as<double>(), p.w_D.as<double>(), bD);
        OSHT_HIP(hipGetLastError());
      }
      gemm_tasks_launch(p, bt + tp[1], tp[2] - tp[1], GemmRole::Correction, "apply_forward_correction", st);
    }
  }
  ProfScope ps(p.prof, "slots_to_coef", st);
  launch_fwd_scatter(p, p.w_Y.as<double>(), flm, B, st, real_maps);
}

bool fwd_blocks_fit(Plan& p, int b) {
  build_fwd_blocks(p, b);
  const size_t need = sizeof(double) * ((size_t)p.fb.max_unk * p.fb.cpw + p.fb.max_w) +
                      sizeof(int32_t) * (p.fb.max_w + p.fb.max_unk + 1);
  return need <= (size_t)p.fb.lds_limit || b == 1;
}

namespace {

__global__ void tune_fill_kernel(double* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (double)((i * 2654435761ll) & 1023) / 512.0 - 1.0;
}

std::string tune_path(const Plan& p) {
  if (p.cache_dir.empty()) return "";
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p.device) != hipSuccess) return "";
  std::string arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ':' || c == '/' || c == ' ') c = '_';
  return p.cache_dir + "/tune_fwd_" + arch + "_L" + std::to_string(p.L) + "_s" + std::to_string(p.spin) + "_p" +
         std::to_string((p.fp32 ? 1 : 0) + (p.fp32_fwd ? 2 : 0) + 4 * p.oz) + ".txt";
}

}  // namespace

void autotune(Plan& p) {
  const std::string path = tune_path(p);
  int best_b = -1, best_c = -1, best_fv = 0, best_iv = 0;
  if (!path.empty()) {
    if (FILE* fp = std::fopen(path.c_str(), "r")) {
      if (std::fscanf(fp, "%d %d %d %d", &best_b, &best_c, &best_fv, &best_iv) != 4 || best_fv < 0 ||
          best_fv >= kGemmVars || best_iv < 0 || best_iv >= kGemmVars)
        best_b = best_c = -1;
      std::fclose(fp);
    }
  }
  if (best_b < 1 || best_c < 1) {
    best_fv = best_iv = 0;
    const int64_t Bt = p.spin == 0 ? 16 : 8;
    const int64_t n = 2 * (int64_t)p.L * p.L * Bt;
    DevBuf in, out;
    in.alloc(sizeof(double) * n);
    out.alloc(sizeof(double) * n);
    hipLaunchKernelGGL(tune_fill_kernel, dim3(1024), dim3(256), 0, 0, in.as<double>(), n);
    OSHT_HIP(hipGetLastError());
    hipEvent_t e0, e1;
    OSHT_HIP(hipEventCreate(&e0));
    OSHT_HIP(hipEventCreate(&e1));
    const bool prof = p.prof.enabled;
    p.prof.enabled = false;
    // three calls after a warm one, between events on the null stream
    auto time3 = [&](auto&& call) {
      call();
      OSHT_HIP(hipEventRecord(e0, 0));
      for (int r = 0; r < 3; ++r) call();
      OSHT_HIP(hipEventRecord(e1, 0));
      OSHT_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      OSHT_HIP(hipEventElapsedTime(&ms, e0, e1));
      return ms;
    };
    float best_ms = 1e30f;
    for (int fv = 0; fv < kGemmVars; ++fv) {
      p.gvar_fwd = fv;
      for (int cpw : {1, 2, 4}) {
        for (int b : {8, 12, 16, 24, 32, 48, 64}) {
          if (b > p.L) continue;
          p.fb.cpw = cpw;
          if (!fwd_blocks_fit(p, b) && b > 1) continue;
          invalidate_tables(p);
          const float ms = time3([&] { run_forward(p, in.as<double>(), out.as<double>(), Bt, 0); });
          if (ms < best_ms) { best_ms = ms; best_b = b; best_c = cpw; best_fv = fv; }
        }
      }
    }
    float best_inv = 1e30f;
    if (p.oz == 0) {  // the int8 inverse apply has a shape of its own
      for (int iv = 0; iv < kGemmVars; ++iv) {
        p.gvar_inv = iv;
        const float ms = time3([&] { run_inverse(p, out.as<double>(), in.as<double>(), Bt, 0); });
        if (ms < best_inv) { best_inv = ms; best_iv = iv; }
      }
    }
    p.prof.enabled = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    OSHT_HIP(hipDeviceSynchronize());
    if (!path.empty() && best_b > 0) {
      const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
      if (FILE* fp = std::fopen(tmp.c_str(), "w")) {
        std::fprintf(fp,
                     "%d %d %d %d\n# forward block levels, delta-solve columns per workgroup, forward-apply and "
                     "inverse-apply stream shapes (%.3f ms for 3 forwards, %.3f ms for 3 inverses)\n",
                     best_b, best_c, best_fv, best_iv, best_ms, p.oz == 0 ? best_inv : 0.f);
        if (std::fclose(fp) == 0) std::rename(tmp.c_str(), path.c_str());
        else std::remove(tmp.c_str());
      }
    }
  }
  p.gvar_fwd = best_fv;
  p.gvar_inv = best_iv;
  if (best_b < 1) return;
  p.fb.cpw = best_c;
  if (!fwd_blocks_fit(p, best_b)) {
    p.fb.cpw = 2;
    int b = 32;
    while (!fwd_blocks_fit(p, b) && b > 1) b = std::max(1, b * 3 / 4);
  }
  invalidate_tables(p);
  p.w_X.release();
  p.w_Y.release();
  p.w_H.release();
  p.w_D.release();
}

void run_forward_adjoint_blocked(Plan& p, const double* flmbar, double* fbar, int64_t B, hipStream_t st) {
  ensure_workspace(p, B);
  const Geo g = geo(p, B);
  const FwdBlocks& fb = p.fb;
  const int bD = std::max(fb.b, 1);
  const int64_t nD = (int64_t)p.nslots * bD * g.ncols;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(nD, 256), 4096)), dim3(256), 0, st,
                     p.w_D.as<double>(), nD);
  OSHT_HIP(hipGetLastError());
  OSHT_HIP(hipFuncSetAttribute((const void*)eps_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                fb.lds_limit));
  const int nblk = (int)fb.q0.size();
  const GemmTask* at = p.tab->d_atask.as<GemmTask>();
  double* H = p.w_H.as<double>();
  for (int blk = nblk - 1; blk >= 0; --blk) {  // ascending orders
    const int ns = fb.slot_ptr[blk + 1] - fb.slot_ptr[blk];
    const int32_t* sl = fb.d_slot_list.as<int32_t>() + fb.slot_ptr[blk];
    const dim3 grid((unsigned)ceil_div((int64_t)p.L * g.ncols, 256), ns);
    hipLaunchKernelGGL(fadj_block_gather_kernel, grid, dim3(256), 0, st, g, p.d_slots.as<Slot>(), sl, fb.q0[blk], flmbar,
                       H, p.w_X.as<double>());
    OSHT_HIP(hipGetLastError());
    const int* tp = &p.tab->h_atask_ptr[2 * blk];
    gemm_tasks_launch(p, at + tp[0], tp[1] - tp[0], GemmRole::Adjoint, "apply_forward_adjoint", st);
    const int u0 = fb.unk_ptr[blk], nu = fb.unk_ptr[blk + 1] - u0;
    if (nu > 0) {
      const int lv0 = fb.lev_blk_ptr[blk], lv1 = fb.lev_blk_ptr[blk + 1];
      const int64_t nw = fb.wt_ptr[u0 + nu] - fb.wt_ptr[u0];
      const int cpw = fb.cpw;
      const size_t lds = sizeof(double) * ((size_t)nu * cpw + nw) + sizeof(int32_t) * (nw + nu + 1);
      hipLaunchKernelGGL(eps_solve_kernel, dim3((unsigned)ceil_div(2 * B, cpw)), dim3(512), lds, st, g, u0, nu,
                         lv1 - lv0 - 1, cpw, fb.q0[blk], fb.d_lev_ptr.as<int32_t>() + lv0, fb.d_unk_slot.as<int32_t>(),
                         fb.d_unk_r.as<int32_t>(), fb.d_unk_m.as<int32_t>(), fb.d_src_ptr.as<int32_t>(),
                         fb.d_src_slot.as<int32_t>(), fb.d_src_m.as<int32_t>(), fb.d_wt_ptr.as<int64_t>(),
                         fb.d_wt_row.as<int32_t>(), fb.d_wt_val.as<double>(), p.w_Y.as<double>(), p.w_D.as<double>(),
                         bD);
      OSHT_HIP(hipGetLastError());
      gemm_tasks_launch(p, at + tp[1], tp[2] - tp[1], GemmRole::Adjoint, "apply_forward_adjoint_correction", st);
    }
    hipLaunchKernelGGL(fadj_block_scatter_kernel, dim3((unsigned)ceil_div((int64_t)p.L * g.ncols, 256), ns), dim3(256),
                       0, st, g, p.d_slots.as<Slot>(), sl, p.w_Y.as<double>(), H);
    OSHT_HIP(hipGetLastError());
  }
  launch_ring_synthesis(p, H, 1, fbar, B, st);
}

}  // namespace osht
