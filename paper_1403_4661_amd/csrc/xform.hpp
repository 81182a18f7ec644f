// Device-side helpers shared by the transform kernels (transform.hip,
// sweep.hip): slot-column decoding and alias addressing.
#pragma once

#include "common.hpp"

namespace osht {

struct Geo {
  int L, s, B, ncols;
};

__device__ __forceinline__ int pmod(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
}

// decode a slot column into (sgn, map, part) and the signed order
__device__ __forceinline__ void decode_col(const Geo& g, const Slot& sl, int col, int& sgn, int& b, int& part, int& m) {
  if (g.s == 0) {
    sgn = col / (2 * g.B);
    const int r = col - sgn * 2 * g.B;
    b = r >> 1;
    part = r & 1;
    m = sgn ? -sl.m : sl.m;
  } else {
    sgn = 0;
    b = col >> 1;
    part = col & 1;
    m = sl.m;
  }
}

// Y-buffer location of G'_{m'}(theta_k) for the forward pass (the bottom
// rows of the slot of order m'), for map b / part.
__device__ __forceinline__ int64_t alias_index(const Geo& g, const Slot* __restrict__ slots, int mp, int k, int b, int part) {
  int slot, col;
  if (g.s == 0) {
    slot = mp < 0 ? -mp : mp;
    col = (mp < 0 ? 2 * g.B : 0) + 2 * b + part;
  } else {
    slot = mp + g.L - 1;
    col = 2 * b + part;
  }
  const int amp = mp < 0 ? -mp : mp;
  const int K = g.L - (amp > (g.s < 0 ? -g.s : g.s) ? amp : (g.s < 0 ? -g.s : g.s));  // L - max(|m'|, |s|)
  (void)slots;
  return ((int64_t)slot * g.L + K + k) * g.ncols + col;
}


// GEMM directions; kFwdAlias / kCorrAlias carry the alias rows of Q_m
// separately in FP32 plans (empty otherwise).
// kFadjCorr: the blocked forward adjoint's correction Z_m -= Q_m^T[:, alias rows of the block] E_m.
enum { kInv = 0, kFwd = 1, kIadj = 2, kFadj = 3, kCorr = 4, kFwdAlias = 5, kCorrAlias = 6, kFadjCorr = 7, kNumDir = 8 };

void ensure_workspace(Plan& p, int64_t B);
// real_maps > 0: flm holds real_maps real maps (two per complex map of the batch B)
void launch_fwd_scatter(const Plan& p, const double* Y, double* flm, int64_t B, hipStream_t st, int64_t real_maps = 0);
void gemm_tasks_launch(Plan& p, const GemmTask* d_tasks, int count, GemmRole role, const char* prof_name,
                       hipStream_t st);

inline Geo geo(const Plan& p, int64_t B) { return Geo{p.L, p.spin, (int)B, (int)(p.ncols_per_map * B)}; }

}  // namespace osht
