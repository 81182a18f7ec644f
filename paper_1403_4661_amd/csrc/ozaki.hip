// Inverse order-wise apply Y_m = A_m X_m as exact integer products of
// int8 splits (the split-and-sum idea of Ozaki, Ogita, Oishi and Rump for
// error-free matrix products, carried out on the int8 matrix cores).
//
// Each FP64 operand is written as a sum of S signed 7-bit digits under a
// power-of-two scale: row i of A_m (ring i) with exponent e_i,
//     A[i, k] = 2^{e_i} sum_{p<S} a_p[i, k] 2^{-7(p+1)} + O(2^{e_i - 7S}),
// column c of X_m (one map, real or imaginary part, one sign of m) with
// exponent f_c likewise (digits b_q), where |A[i, k]| < 2^{e_i} and the digits
// come from repeated truncation: t = trunc(128 r), r <- 128 r - t (exact in
// FP64), so every digit lies in [-127, 127].  The product keeps the digit
// pairs p + q < S:
//     Y[i, c] = 2^{e_i + f_c} sum_{d<S} 2^{-7(d+2)} D_d[i, c],
//     D_d = sum_{p+q=d} a_p b_q   (int32: at most S * 127^2 * K < 2^31),
// each D_d accumulated exactly by v_mfma_i32_16x16x64_i8 and scaled and
// summed in FP64 at the end.  The error falls by about 2^7 per digit (CPU
// emulation at L = 256: 2e-8 with 5 digits, 2e-10 with 6, 2e-12 with 7,
// relative to max |f|); FP32 operands give 4e-8.
//
// Layouts.  A digits (plan): per slot, plane p at offA8 + p * Mp * Kp, Mp = L
// rounded up to 64, Kp = K rounded up to 64, zero padded, in 1 KB blocks of
// 16 rows x 64 k (k contiguous within a row): block (i / 16, k / 64) at
// ((i / 16) (Kp / 64) + k / 64) * 1024, entry (i % 16) * 64 + k % 64, so one
// wave's load of a k step (16 rows x 64 bytes) is one contiguous kilobyte;
// e_i at Aexp[slot * Mp + i].  Digit row i is ring rowmap[i], the rings in
// ascending sin(theta), and a task starts its k loop at its row tile's
// first k step holding a nonzero digit (GemmTask::pad).  X digits (per
// call): per slot, plane q at
// slot * S * Np * Kx + q * Np * Kx, Np = the slot columns rounded up to 64,
// Kx = L rounded up to 64, in 4 KB blocks of 64 columns x 64 k (k contiguous
// within a column): block (c / 64, k / 64) at ((c / 64) (Kx / 64) + k / 64)
// * 4096, entry (c % 64) * 64 + k % 64 -- a workgroup's k step of B is one
// contiguous block; f_c at Xexp[slot * Np + c].
//
// GEMM: one workgroup (4 waves) per 64 x 64 tile of Y; wave w owns rows
// [16w, 16w + 16) and all 64 columns as four 16 x 16 blocks with S int32
// accumulators each (one per digit sum d).  Per 64-deep k step, each lane
// loads its 16-byte A chunk of every digit plane from HBM into registers
// (one step ahead; every A byte is read once), and the workgroup loads the
// step's B digits (S planes x 64 columns x 64 bytes, from L2) into a
// double-buffered LDS tile.  MFMA operands: lane l supplies row (l % 16) of A
// and column (l % 16) of B, digits k = 16 (l / 16) .. +15 of the step (any
// k order shared by A and B gives the same sum); accumulator v of lane l
// holds D[4 (l / 16) + v][l % 16].  LDS columns of 64 bytes hold their four
// 16-byte chunks XOR-swizzled by (column / 4) % 4, so the 16 lanes of a k
// group read 16 distinct bank quads.

#include <algorithm>
#include <climits>
#include <cstdlib>

#include "host_util.hpp"
#include "xform.hpp"

namespace osht {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kOzTile = 64;

template <int S>
__device__ __forceinline__ void digits(double r, int8_t* out) {
#pragma unroll
  for (int p = 0; p < S; ++p) {
    const double t = trunc(r * 128.0);
    out[p] = (int8_t)(int)t;
    r = r * 128.0 - t;
  }
}

// exponent e with |v| < 2^e (0 for v = 0)
// Offset of digit (column c, k) within one plane of the blocked X layout.
__device__ __forceinline__ int64_t xblk(int c, int k, int Kx) {
  return ((int64_t)(c >> 6) * (Kx >> 6) + (k >> 6)) * 4096 + (c & 63) * 64 + (k & 63);
}

__device__ __forceinline__ int exp_above(double v) {
  int e = 0;
  if (v != 0.0) (void)frexp(v, &e);
  return e;
}

// Plan: A_m (FP64, column-major L x K, leading dimension ldA) -> digits.
// Digit row r holds ring rowmap[r].  One workgroup per (64-row tile, slot).
// Thread t handles row t / 4 and, in every 64 columns, the 16 columns
// 16 (t % 4) .. +15: it takes the row maximum over them, then digits them
// and stores each plane's 16 bytes as one vector, so four consecutive
// threads write 64 contiguous bytes.  The tile's first 64-deep k-step with
// a nonzero digit goes to kstart[slot * gridDim.x + tile] (Kp / 64 when
// every digit of the tile is zero).
template <int S>
__global__ __launch_bounds__(256) void oz_split_a_kernel(const Slot* __restrict__ slots, const double* __restrict__ A,
                                                         int L, int Mp, const int64_t* __restrict__ offA8,
                                                         const int32_t* __restrict__ rowmap, int8_t* __restrict__ A8,
                                                         int32_t* __restrict__ Aexp, int32_t* __restrict__ kstart) {
  __shared__ double red[64][4];
  __shared__ int first;
  const int slot = blockIdx.y, m0 = blockIdx.x * 64;
  const Slot sl = slots[slot];
  const int Kp = (sl.K + 63) / 64 * 64;
  const int t = threadIdx.x, row = t >> 2, j = t & 3;
  const int r = m0 + row;
  const double* Ac = A + sl.offA;
  if (t == 0) first = Kp / 64;
  double mx = 0.0;
  // out-of-range entries load a valid one and are dropped by a select, so
  // that the 16 loads of a step are issued together
  const int rr = rowmap[min(r, L - 1)];
  if (r < L) {
    for (int k0 = 16 * j; k0 < sl.K; k0 += 64) {
      double v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = fabs(Ac[rr + (int64_t)min(k0 + i, sl.K - 1) * sl.ldA]);
#pragma unroll
      for (int i = 0; i < 16; ++i) mx = fmax(mx, k0 + i < sl.K ? v[i] : 0.0);
    }
  }
  red[row][j] = mx;
  __syncthreads();
  const int e = exp_above(fmax(fmax(red[row][0], red[row][1]), fmax(red[row][2], red[row][3])));
  if (j == 0) Aexp[(int64_t)slot * Mp + r] = e;
  int8_t* out = A8 + offA8[slot];
  for (int k0 = 16 * j; k0 < Kp; k0 += 64) {
    v4i w[S];
#pragma unroll
    for (int p = 0; p < S; ++p) w[p] = v4i{0, 0, 0, 0};
    double av[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) av[i] = Ac[rr + (int64_t)min(k0 + i, sl.K - 1) * sl.ldA];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int k = k0 + i;
      const double v = (r < L && k < sl.K) ? av[i] : 0.0;
      int8_t dg[S];
      digits<S>(ldexp(v, -e), dg);
#pragma unroll
      for (int p = 0; p < S; ++p) w[p][i >> 2] |= (int)(uint8_t)dg[p] << (8 * (i & 3));
    }
#pragma unroll
    for (int p = 0; p < S; ++p)
      *reinterpret_cast<v4i*>(out + (int64_t)p * Mp * Kp + ((int64_t)(r >> 4) * (Kp >> 6) + (k0 >> 6)) * 1024 +
                              (r & 15) * 64 + (k0 & 63)) = w[p];
    bool nz = false;
#pragma unroll
    for (int p = 0; p < S; ++p) nz = nz || (w[p][0] | w[p][1] | w[p][2] | w[p][3]) != 0;
    if (nz) atomicMin(&first, k0 >> 6);
  }
  __syncthreads();
  if (t == 0) kstart[(int64_t)slot * gridDim.x + blockIdx.x] = first;
}

// Per call: slot-layout right-hand sides X[slot][row][col] (FP64, rows
// l - l0 < K, ncols columns) -> per-column exponents and digits, in two
// launches over (slot, 256-row chunk) workgroups: the column maxima of each
// chunk (as exponents, combined by atomicMax into Xexp, which starts at
// INT_MIN), then the digits.  Thread t handles column c0 + t / 4 and rows
// 16 (t % 4) + 64 i .. +15 of the chunk; each plane's 16 bytes are stored as
// one vector, so four consecutive threads write 64 contiguous bytes.
constexpr int kSplitRows = 256;

__global__ __launch_bounds__(256) void oz_fill_kernel(int32_t* __restrict__ x, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}

__global__ __launch_bounds__(256) void oz_colexp_kernel(const Slot* __restrict__ slots, const double* __restrict__ X,
                                                        int L, int ncols, int Np, int32_t* __restrict__ Xexp) {
  __shared__ double red[64][4];
  const int slot = blockIdx.x, rc = blockIdx.y * kSplitRows;
  const int K = slots[slot].K;
  if (rc >= K) return;  // uniform
  const int rend = min(K, rc + kSplitRows);
  const int t = threadIdx.x, cl = t >> 2, j = t & 3;
  const double* Xs = X + (int64_t)slot * L * ncols;
  for (int c0 = 0; c0 < ncols; c0 += 64) {
    const int c = c0 + cl;
    double mx = 0.0;
    if (c < ncols) {
      for (int r0 = rc + 16 * j; r0 < rend; r0 += 64) {
        // rows past the end load row rend - 1 again and are dropped by the
        // select: a load under a branch is waited for before the next one
        double v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = fabs(Xs[(int64_t)min(r0 + i, rend - 1) * ncols + c]);
#pragma unroll
        for (int i = 0; i < 16; ++i) mx = fmax(mx, r0 + i < rend ? v[i] : 0.0);
      }
    }
    red[cl][j] = mx;
    __syncthreads();
    if (j == 0 && c < ncols) {
      const double m = fmax(fmax(red[cl][0], red[cl][1]), fmax(red[cl][2], red[cl][3]));
      if (m > 0.0) atomicMax(&Xexp[(int64_t)slot * Np + c], exp_above(m));
    }
    __syncthreads();  // red is rewritten by the next column chunk
  }
}

template <int S>
__global__ __launch_bounds__(256) void oz_split_x_kernel(const Slot* __restrict__ slots, const double* __restrict__ X,
                                                         int L, int ncols, int Np, int Kx, int8_t* __restrict__ X8,
                                                         const int32_t* __restrict__ Xexp) {
  const int slot = blockIdx.x, rc = blockIdx.y * kSplitRows;
  const int K = slots[slot].K;
  const int Kp = (K + 63) / 64 * 64;
  if (rc >= Kp) return;  // uniform
  const int rend = min(Kp, rc + kSplitRows);
  const int t = threadIdx.x, cl = t >> 2, j = t & 3;
  const double* Xs = X + (int64_t)slot * L * ncols;
  int8_t* out = X8 + (int64_t)slot * S * Np * Kx;
  for (int c0 = 0; c0 < Np; c0 += 64) {
    const int c = c0 + cl;
    int e = c < ncols ? Xexp[(int64_t)slot * Np + c] : 0;
    if (e == INT_MIN) e = 0;  // an all-zero column
    const int cc = min(c, ncols - 1);  // padding columns load column ncols - 1 and drop it
    for (int r0 = rc + 16 * j; r0 < rend; r0 += 64) {
      v4i w[S];
#pragma unroll
      for (int p = 0; p < S; ++p) w[p] = v4i{0, 0, 0, 0};
      // all 16 loads issued before any is used (a load under a branch is
      // waited for before the next one); rows past K load row K - 1 and are
      // dropped by the select
      double xv[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) xv[i] = Xs[(int64_t)min(r0 + i, K - 1) * ncols + cc];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = r0 + i;
        const double v = (c < ncols && r < K) ? xv[i] : 0.0;
        int8_t dg[S];
        digits<S>(ldexp(v, -e), dg);
#pragma unroll
        for (int p = 0; p < S; ++p) w[p][i >> 2] |= (int)(uint8_t)dg[p] << (8 * (i & 3));
      }
#pragma unroll
      for (int p = 0; p < S; ++p)
        *reinterpret_cast<v4i*>(out + (int64_t)p * Np * Kx + xblk(c, r0, Kx)) = w[p];
    }
  }
}

// The exponents and digits of the right-hand side in one pass: one
// workgroup per (slot, CW columns), thread (column c = t % CW, q = t / CW)
// holding rows [16 (q + NQ i), +16), i < NCH, NQ = 256 / CW, in registers,
// so 16 NQ NCH rows at most (CW = 16, NCH = 4: L <= 1024; CW = 8, NCH = 4:
// L <= 2048).  CW = 16 reads whole 128-byte row pieces (CW = 8 fetched each
// line twice).  The column maximum comes from those registers and an LDS
// reduction, then the same registers are split, so X is read from HBM once
// (the two-kernel path above reads it twice).  Exponents and digits are
// those of that path: an all-zero column stores exponent 0.
template <int S, int CW, int NCH>
__global__ __launch_bounds__(256) void oz_xsplit_kernel(const Slot* __restrict__ slots, const double* __restrict__ X,
                                                        int L, int ncols, int Np, int Kx, int8_t* __restrict__ X8,
                                                        int32_t* __restrict__ Xexp) {
  constexpr int NQ = 256 / CW;
  __shared__ double red[NQ][CW];
  __shared__ int ecol[CW];
  const int slot = blockIdx.x, cl = threadIdx.x % CW, q = threadIdx.x / CW;
  const int c = blockIdx.y * CW + cl;
  const int K = slots[slot].K, Kp = (K + 63) / 64 * 64;
  const double* Xs = X + (int64_t)slot * L * ncols;
  const int cc = min(c, ncols - 1);  // padding columns load column ncols - 1 and drop it
  double v[NCH][16];
  // every load issued before any is used; rows past K load row K - 1
#pragma unroll
  for (int i = 0; i < NCH; ++i)
#pragma unroll
    for (int j = 0; j < 16; ++j) v[i][j] = Xs[(int64_t)min(16 * (q + NQ * i) + j, K - 1) * ncols + cc];
  double mx = 0.0;
#pragma unroll
  for (int i = 0; i < NCH; ++i)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const bool ok = c < ncols && 16 * (q + NQ * i) + j < K;
      v[i][j] = ok ? v[i][j] : 0.0;
      mx = fmax(mx, fabs(v[i][j]));
    }
  red[q][cl] = mx;
  __syncthreads();
  if (q == 0) {
    double m = 0.0;
    for (int i = 0; i < NQ; ++i) m = fmax(m, red[i][cl]);
    const int e = exp_above(m);
    ecol[cl] = e;
    Xexp[(int64_t)slot * Np + c] = e;
  }
  __syncthreads();
  const int e = ecol[cl];
  int8_t* out = X8 + (int64_t)slot * S * Np * Kx;
#pragma unroll
  for (int i = 0; i < NCH; ++i) {
    const int r0 = 16 * (q + NQ * i);
    if (r0 >= Kp) continue;
    v4i w[S];
#pragma unroll
    for (int p = 0; p < S; ++p) w[p] = v4i{0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      int8_t dg[S];
      digits<S>(ldexp(v[i][j], -e), dg);
#pragma unroll
      for (int p = 0; p < S; ++p) w[p][j >> 2] |= (int)(uint8_t)dg[p] << (8 * (j & 3));
    }
#pragma unroll
    for (int p = 0; p < S; ++p) *reinterpret_cast<v4i*>(out + (int64_t)p * Np * Kx + xblk(c, r0, Kx)) = w[p];
  }
}

// Global-memory views of descriptor pointers (plain pointers compile to flat
// accesses, which also count in lgkmcnt and so would stall every LDS wait).
typedef __attribute__((address_space(1))) const v4i* gv4i_ptr;
typedef __attribute__((address_space(1))) const int32_t* gi32_ptr;
typedef __attribute__((address_space(1))) double* gf64_ptr;

template <int S>
__device__ __forceinline__ void oz_load(gv4i_ptr src, int64_t plane, v4i* r) {
#pragma unroll
  for (int p = 0; p < S; ++p) r[p] = *(gv4i_ptr)((__attribute__((address_space(1))) const int8_t*)src + p * plane);
}

// All loads of the k loop go to registers (none straight to LDS): the
// compiler then counts them in order and waits only for what each step
// needs.  A: wave w loads its own 16 rows (each A byte is read once);
// B: every thread loads one 16-byte chunk of one column per digit plane and
// stores it to a double-buffered LDS tile, from which all four waves read.
// PF: k steps of A held in flight per wave (registers), 1 or 2.
template <int S, int PF>
__global__ __launch_bounds__(256) void oz_apply_kernel(const OzDesc* __restrict__ descs,
                                                       const GemmTask* __restrict__ tasks) {
  __shared__ __align__(16) char bs[2][S][64 * 64];
  // task order as in the streaming GEMM: runs of 16 consecutive tasks (the
  // row tiles of one slot, which share its right-hand side) on one XCD
  constexpr int C = 16, RND = 8 * C;
  const int G = gridDim.x, bid = blockIdx.x, base = (bid / RND) * RND, pp = bid - base;
  int ti;
  if (base + RND <= G) {
    ti = base + (pp & 7) * C + (pp >> 3);
  } else {
    const int Sz = G - base, q = Sz >> 3, r = Sz & 7, x = pp & 7, l = pp >> 3;
    ti = base + (x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l);
  }
  const GemmTask tk = tasks[ti];
  const OzDesc d = descs[tk.desc];
  const int m0 = tk.mt * kOzTile, n0 = tk.nt * kOzTile;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int li = lane & 15, kq = lane >> 4;
  // k-steps [0, tk.pad) of this row tile hold only zero digits of A (its
  // rings' negligible Legendre values): they add nothing and are skipped
  const int nk = d.Kp / 64 - tk.pad;
  // this lane's A chunk: row m0 + 16 wave + li, bytes [16 kq, 16 kq + 16) of
  // each 64-deep step, in the 1 KB block of its 16 rows (steps 1 KB apart)
  gv4i_ptr asrc = (gv4i_ptr)(d.A + ((int64_t)((m0 >> 4) + wave) * (d.Kp / 64) + tk.pad) * 1024 + li * 64 + 16 * kq);
  // this thread's B chunk: column n0 + (t >> 2), bytes [16 (t & 3), +16)
  const int bc = t >> 2, bch = t & 3;
  // (steps 4 KB apart in the column tile's blocks)
  gv4i_ptr bsrc = (gv4i_ptr)(d.X + xblk(n0 + bc, 16 * bch + 64 * tk.pad, d.ldX));
  const int bpos = bc * 64 + 16 * (bch ^ ((bc >> 2) & 3));
  v4i acc[4][S];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int dd = 0; dd < S; ++dd) acc[cb][dd] = v4i{0, 0, 0, 0};
  // the epilogue's row and column exponents, loaded before the k loop
  // (clamped indices; the unused ones are dropped): guarded one by one in
  // the epilogue, each was waited for in turn after the last product
  int ear[4], xe[4], ring[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) ear[v] = ((gi32_ptr)d.ea)[min(m0 + 16 * wave + 4 * kq + v, d.M - 1)];
#pragma unroll
  for (int v = 0; v < 4; ++v) ring[v] = ((gi32_ptr)d.rowmap)[min(m0 + 16 * wave + 4 * kq + v, d.M - 1)];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) xe[cb] = ((gi32_ptr)d.xe)[min(n0 + cb * 16 + li, d.N - 1)];
  v4i a[S], an[S], an2[S], an3[S], bt[S];
  if (nk > 0) {
    oz_load<S>(asrc, d.planeA, a);
    if (PF >= 2) oz_load<S>(asrc + min(1, nk - 1) * 64, d.planeA, an);
    if (PF >= 3) oz_load<S>(asrc + min(2, nk - 1) * 64, d.planeA, an2);
    oz_load<S>(bsrc, d.planeX, bt);
#pragma unroll
    for (int p = 0; p < S; ++p) *reinterpret_cast<v4i*>(&bs[0][p][bpos]) = bt[p];
  }
  for (int kt = 0; kt < nk; ++kt) {
    // A digits PF steps ahead and the next step's B digits (past the last
    // step the last one is reloaded, so every path issues the same loads)
    oz_load<S>(asrc + min(kt + PF, nk - 1) * 64, d.planeA, PF == 3 ? an3 : PF == 2 ? an2 : an);
    oz_load<S>(bsrc + min(kt + 1, nk - 1) * 256, d.planeX, bt);
    __syncthreads();  // B tile of step kt stored by every thread
    const char* st = bs[kt & 1][0];
    // B fragments of column block cb + 1 are read from LDS while the
    // products of block cb run
    v4i bf[2][S];
    auto read_b = [&](int cb, v4i* dst) {
      const int c = cb * 16 + li;
      const int off = c * 64 + 16 * (kq ^ ((c >> 2) & 3));
#pragma unroll
      for (int q = 0; q < S; ++q) dst[q] = *reinterpret_cast<const v4i*>(st + q * 4096 + off);
    };
    read_b(0, bf[0]);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      if (cb + 1 < 4) read_b(cb + 1, bf[(cb + 1) & 1]);
#pragma unroll
      for (int q = 0; q < S; ++q)
#pragma unroll
        for (int p = 0; p + q < S; ++p)
          acc[cb][p + q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[p], bf[cb & 1][q], acc[cb][p + q], 0, 0, 0);
    }
    // the other buffer was last read in step kt - 1, which every wave has
    // finished (it passed this step's barrier)
#pragma unroll
    for (int p = 0; p < S; ++p) *reinterpret_cast<v4i*>(&bs[(kt + 1) & 1][p][bpos]) = bt[p];
#pragma unroll
    for (int p = 0; p < S; ++p) {
      a[p] = an[p];
      if (PF >= 2) an[p] = an2[p];
      if (PF >= 3) an2[p] = an3[p];
    }
  }
  gf64_ptr Cg = (gf64_ptr)d.C;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int col = n0 + cb * 16 + li;
    if (col >= d.N) continue;
    int fe = xe[cb];
    if (fe == INT_MIN) fe = 0;  // an all-zero column (its digits and products are zero)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = m0 + 16 * wave + 4 * kq + v;
      if (r < d.M) {
        const int e = ear[v] + fe;
        double y = 0.0;
#pragma unroll
        for (int dd = 0; dd < S; ++dd) y += ldexp((double)acc[cb][dd][v], e - 7 * (dd + 2));
        Cg[(int64_t)ring[v] * d.ldc + col] = y;
      }
    }
  }
}

// A prefetch depth (k steps held in registers per wave): two steps measured
// no faster than one with 6 digits, and 8 digits have no registers to spare.
template <int S> struct OzCfg { static constexpr int PF = 1; };

template <int S>
void oz_launch_apply(const OzDesc* d_desc, const GemmTask* d_task, int ntask, hipStream_t st, hipEvent_t e0,
                     hipEvent_t e1) {
  const void* fn = (const void*)oz_apply_kernel<S, OzCfg<S>::PF>;
  if (e0) {
    void* args[] = {(void*)&d_desc, (void*)&d_task};
    OSHT_HIP(hipExtLaunchKernel(fn, dim3(ntask), dim3(256), args, 0, st, e0, e1, 0));
  } else {
    hipLaunchKernelGGL((oz_apply_kernel<S, OzCfg<S>::PF>), dim3(ntask), dim3(256), 0, st, d_desc, d_task);
  }
  OSHT_HIP(hipGetLastError());
}

}  // namespace

int oz_x_cols(const Plan& p, int64_t B) { return (int)ceil_div(p.ncols_per_map * B, kOzTile) * kOzTile; }
int oz_x_ld(const Plan& p) { return (int)ceil_div(p.L, kOzTile) * kOzTile; }

void build_oz_planes(Plan& p) {
  const int S = p.oz;
  const int Mp = (int)ceil_div(p.L, kOzTile) * kOzTile;
  std::vector<int64_t> off(p.nslots);
  int64_t tot = 0;
  for (int i = 0; i < p.nslots; ++i) {
    off[i] = tot;
    tot += (int64_t)S * Mp * (ceil_div(p.slots[i].K, kOzTile) * kOzTile);
  }
  p.oz_offA8 = off;
  upload(p.d_ozoff, off);
  // digit rows: the rings in ascending sin(theta) (ties by ring index).  A
  // ring's Legendre values are negligible below degree ~|m| / sin(theta)
  // and decay from there towards the pole, so rings of similar sin(theta)
  // share their run of all-zero leading k-steps
  std::vector<int32_t> rowmap(p.L);
  {
    std::vector<double> sn(p.L);
    for (int k = 0; k < p.L; ++k) ring_trig(p.L, p.numer[k], nullptr, &sn[k], nullptr, nullptr);
    for (int k = 0; k < p.L; ++k) rowmap[k] = k;
    std::stable_sort(rowmap.begin(), rowmap.end(), [&](int32_t a, int32_t b) { return sn[a] < sn[b]; });
  }
  upload(p.d_ozrow, rowmap);
  p.oz_rowmap = rowmap;
  const int tiles = Mp / kOzTile;
  p.d_A8.alloc((size_t)std::max<int64_t>(tot, 1));
  p.d_Aexp.alloc(sizeof(int32_t) * (size_t)p.nslots * Mp);
  p.d_ozkstart.alloc(sizeof(int32_t) * (size_t)p.nslots * tiles);
  const dim3 grid((unsigned)tiles, (unsigned)p.nslots);
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, grid, dim3(256), 0, 0, p.d_slots.as<Slot>(), p.d_A.as<double>(), p.L, Mp,
                       p.d_ozoff.as<int64_t>(), p.d_ozrow.as<int32_t>(), p.d_A8.as<int8_t>(), p.d_Aexp.as<int32_t>(),
                       p.d_ozkstart.as<int32_t>());
  };
  if (S == 6) go(oz_split_a_kernel<6>);
  else if (S == 8) go(oz_split_a_kernel<8>);
  else throw Error{OSHT_ENOTSUP, "unsupported number of int8 digits"};
  OSHT_HIP(hipGetLastError());
  OSHT_HIP(hipDeviceSynchronize());
  p.oz_kstart.assign((size_t)p.nslots * tiles, 0);
  OSHT_HIP(hipMemcpy(p.oz_kstart.data(), p.d_ozkstart.p, sizeof(int32_t) * p.oz_kstart.size(), hipMemcpyDeviceToHost));
  // OSHT_OZ_KSKIP=0: every task runs its full k loop (tests compare the two)
  if (const char* e = std::getenv("OSHT_OZ_KSKIP"))
    if (std::atoi(e) == 0) std::fill(p.oz_kstart.begin(), p.oz_kstart.end(), 0);
}

void oz_descs(const Plan& p, int64_t B, const double* Y, int8_t* X8, const int32_t* Xexp, std::vector<OzDesc>& descs,
              std::vector<GemmTask>& tasks) {
  const int S = p.oz;
  const int Mp = (int)ceil_div(p.L, kOzTile) * kOzTile;
  const int ncols = p.ncols_per_map * (int)B, Np = oz_x_cols(p, B), Kx = oz_x_ld(p);
  descs.clear();
  tasks.clear();
  for (int i = 0; i < p.nslots; ++i) {
    const Slot& sl = p.slots[i];
    OzDesc d{};
    const int Kp = (int)ceil_div(sl.K, kOzTile) * kOzTile;
    d.A = p.d_A8.as<int8_t>() + p.oz_offA8[i];
    d.ea = p.d_Aexp.as<int32_t>() + (int64_t)i * Mp;
    d.rowmap = p.d_ozrow.as<int32_t>();
    d.X = X8 + (int64_t)i * S * Np * Kx;
    d.xe = Xexp + (int64_t)i * Np;
    d.C = const_cast<double*>(Y) + (int64_t)i * p.L * ncols;
    d.planeA = (int64_t)Mp * Kp;
    d.planeX = (int64_t)Np * Kx;
    d.M = p.L;
    d.N = ncols;
    d.Kp = Kp;
    d.ldX = Kx;
    d.ldc = ncols;
    descs.push_back(d);
    const int am = std::abs(sl.m);
    for (int a = 0; a < Mp / kOzTile; ++a) {
      // a tile whose rings all lie past this order's ring cut is left out:
      // the fold reads none of its rows
      bool needed = false;
      for (int r = a * kOzTile; r < std::min(p.L, (a + 1) * kOzTile); ++r)
        needed = needed || am < p.h_ring_cut[p.oz_rowmap[r]];
      if (!needed) continue;
      const int k0 = p.oz_kstart[(size_t)i * (Mp / kOzTile) + a];  // leading all-zero k-steps
      for (int c = 0; c < Np / kOzTile; ++c) tasks.push_back(GemmTask{i, a, c, k0});
    }
  }
}

void launch_oz_split_x(const Plan& p, const double* X, int64_t B, int8_t* X8, int32_t* Xexp, hipStream_t st) {
  const int ncols = p.ncols_per_map * (int)B, Np = oz_x_cols(p, B), Kx = oz_x_ld(p);
  if (Kx <= 2048) {  // one pass, a slot's rows of 16 (L <= 1024) or 8 columns in registers
    const int cw = Kx <= 1024 ? 16 : 8;
    const dim3 grid((unsigned)p.nslots, (unsigned)(Np / cw));
    auto go1 = [&](auto kernel) {
      hipLaunchKernelGGL(kernel, grid, dim3(256), 0, st, p.d_slots.as<Slot>(), X, p.L, ncols, Np, Kx, X8, Xexp);
    };
    if (p.oz == 6) cw == 16 ? go1(oz_xsplit_kernel<6, 16, 4>) : go1(oz_xsplit_kernel<6, 8, 4>);
    else cw == 16 ? go1(oz_xsplit_kernel<8, 16, 4>) : go1(oz_xsplit_kernel<8, 8, 4>);
    OSHT_HIP(hipGetLastError());
    return;
  }
  const int64_t ne = (int64_t)p.nslots * Np;
  hipLaunchKernelGGL(oz_fill_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(ne, 256), 1024)), dim3(256), 0, st, Xexp,
                     ne, (int32_t)INT_MIN);
  OSHT_HIP(hipGetLastError());
  const dim3 grid((unsigned)p.nslots, (unsigned)ceil_div(Kx, kSplitRows));
  hipLaunchKernelGGL(oz_colexp_kernel, grid, dim3(256), 0, st, p.d_slots.as<Slot>(), X, p.L, ncols, Np, Xexp);
  OSHT_HIP(hipGetLastError());
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, grid, dim3(256), 0, st, p.d_slots.as<Slot>(), X, p.L, ncols, Np, Kx, X8,
                       static_cast<const int32_t*>(Xexp));
  };
  if (p.oz == 6) go(oz_split_x_kernel<6>);
  else go(oz_split_x_kernel<8>);
  OSHT_HIP(hipGetLastError());
}

void launch_oz_apply(const Plan& p, const OzDesc* d_desc, const GemmTask* d_task, int ntask, hipStream_t st,
                     hipEvent_t e0, hipEvent_t e1) {
  if (ntask <= 0) return;
  if (p.oz == 6) oz_launch_apply<6>(d_desc, d_task, ntask, st, e0, e1);
  else oz_launch_apply<8>(d_desc, d_task, ntask, st, e0, e1);
}

}  // namespace osht
