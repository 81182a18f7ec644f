// Internal declarations shared by the HIP sources of libosht.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/osht.h"

namespace osht {

// ---------------------------------------------------------------- errors
struct Error {
  int code;
  std::string msg;
};

#define OSHT_HIP(call)                                                            \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      throw ::osht::Error{e_ == hipErrorOutOfMemory ? OSHT_ENOMEM : OSHT_EHIP,    \
                          std::string(#call) + ": " + hipGetErrorString(e_)};     \
    }                                                                             \
  } while (0)

#define OSHT_CHECK(cond, code, what)                                              \
  do {                                                                            \
    if (!(cond)) throw ::osht::Error{(code), (what)};                             \
  } while (0)

// Owning device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    OSHT_HIP(hipMalloc(&p, n));
    bytes = n;
  }
  // grows (never shrinks); contents are not preserved
  void reserve(size_t n) {
    if (n > bytes) alloc(n);
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

template <class T>
void upload(DevBuf& d, const std::vector<T>& h) {
  d.alloc(h.size() * sizeof(T));
  if (!h.empty()) OSHT_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

// ---------------------------------------------------------------- plan
// One "slot" per order handled by one matrix.  Spin 0: slot am covers the
// two orders +am and -am (P_{-m} = (-1)^m P_m), RHS columns [+am | -am].
// Spin s != 0: slot = m + L - 1 covers the single signed order m.
struct Slot {
  int32_t m;     // signed order (spin 0: am >= 0)
  int32_t l0;    // first degree max(|m|, |s|)
  int32_t K;     // unknowns L - l0
  int32_t R;     // system rows L - |m| (rings |m| .. L-1)
  int64_t offA;  // A_slot: L x K, column-major, leading dim ldA
  int32_t ldA;
  int32_t ldQ;   // Q_slot: (K + |m|) x R, column-major
  int64_t offQ;
};

// Batched GEMM descriptor: C(MxN) = alpha * A(MxK) * B(KxN) + beta * C,
// element (i, j) of X at X[i * sXr + j * sXc].
struct GemmDesc {
  const void* A;  // double, or float for FP32-matrix plans

  const double* B;
  double* C;
  int64_t sAr, sAc, sBr, sBc, sCr, sCc;
  int32_t M, N, K;
  int32_t fp32;   // A is float (else double)
  double alpha, beta;
  int32_t m_lo;   // rows [m_lo, M) are computed and stored (tiles start at m_lo / 64)
  int32_t b32;    // B is float (else double); GemmRole::ApplyInverse32 only
  int32_t c32;    // C is stored as float (beta must be 0); GemmRole::ApplyInverse32 only
  int32_t pad;
};

struct GemmTask {
  int32_t desc, mt, nt, pad;  // pad: int8 apply tasks, the row tile's leading all-zero k-steps
};

// Inverse apply on int8 digit splits (ozaki.hip): Y = A X for one slot.
struct OzDesc {
  const int8_t* A;     // digit plane 0 of A (row-major, leading dimension Kp); plane p at A + p * planeA
  const int32_t* ea;   // row exponents
  const int32_t* rowmap;  // ring of each digit row (rows sorted by sin theta)
  const int8_t* X;     // digit plane 0 of X (column-major, leading dimension ldX); plane q at X + q * planeX
  const int32_t* xe;   // column exponents
  double* C;           // Y (row-major, leading dimension ldc)
  int64_t planeA, planeX;
  int32_t M, N, Kp, ldX, ldc, pad;
};

// Ring DFT geometry: ring k has n = 2k+1 samples; Bluestein size M_k.
struct RingDesc {
  int32_t n;      // 2k+1
  int32_t logM;   // log2 of the Bluestein FFT size
  int64_t off;    // offset of the chirp spectrum (M complex) in chirp table
};

// Event-pair timing of named kernel launches (see osht_plan_set_profiling).
struct Profiler {
  struct Stat {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    int64_t count = 0;
    double ms = 0.0;
  };
  bool enabled = false;
  std::string only;  // when not empty, the one name that is timed
  bool wants(const char* name) const { return enabled && (only.empty() || only == name); }
  std::vector<std::pair<std::string, Stat>> stats;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  Stat& stat(const char* name);
  void reset();
  void flush(Stat& s);
  ~Profiler();
};

// Blocked forward sweep (built once per plan).  Levels |m| are processed in
// blocks [q0, q1), highest first; the unknowns of block i are the alias rows
// (m, k), q0 <= |m| <= k < q1, that receive aliases from other orders of the
// same block (see sweep.hip).
struct FwdBlocks {
  int b = 1;                                   // levels per block
  std::vector<int32_t> q0, q1;                 // per block
  std::vector<int32_t> slot_ptr, slot_list;    // block -> slots
  std::vector<int32_t> unk_ptr;                // block -> unknowns [u0, u1)
  std::vector<int32_t> lev_blk_ptr, lev_ptr;   // block -> levels -> unknown offsets
  std::vector<int32_t> unk_slot, unk_r, unk_m; // per unknown
  std::vector<int32_t> src_ptr, src_slot, src_row, src_m;
  std::vector<int64_t> w_ptr;                  // per unknown -> W entries
  std::vector<int32_t> w_col;                  // block-local unknown index
  std::vector<int64_t> w_idx;                  // element of d_Q holding the value
  std::vector<int64_t> wt_ptr;                 // per unknown u': W^T entries (u, W_{u,u'}), for the adjoint
  std::vector<int32_t> wt_row;                 // block-local u
  std::vector<int64_t> wt_idx;                 // element of d_Q holding W_{u,u'}
  int kthr = 0;                                // rings k < kthr: wide gather
  std::vector<int32_t> wide_ptr, wide_slot, wide_row;  // block -> (slot, row) pairs of rings k < kthr
  int max_unk = 0;
  int64_t max_w = 0;                           // max W entries in one block
  int cpw = 1;                                 // delta-solve columns per workgroup
  // (I + W)^{-1} of every block with column u repeated for each source of
  // unknown u, column-major with leading dimension minv_ld[blk], at element
  // offset minv_off[blk] of d_minv; the forward then takes delta as one
  // matrix product per block (d_src_yrow: the sources' alias rows)
  bool dense = true;
  std::vector<int64_t> minv_off;
  std::vector<int32_t> minv_ld;
  int lds_limit = 160 * 1024;
  void clear_host() {
    for (auto* v : {&q0, &q1, &slot_ptr, &slot_list, &unk_ptr, &lev_blk_ptr, &lev_ptr, &unk_slot, &unk_r, &unk_m,
                    &src_ptr, &src_slot, &src_row, &src_m, &w_col, &wide_ptr, &wide_slot, &wide_row, &wt_row})
      v->clear();
    w_ptr.clear();
    w_idx.clear();
    wt_ptr.clear();
    wt_idx.clear();
    max_unk = 0;
  }
  DevBuf d_slot_list, d_lev_ptr, d_unk_slot, d_unk_r, d_unk_m, d_src_ptr, d_src_slot, d_src_row, d_src_m,
      d_w_ptr, d_w_col, d_w_val, d_wide_slot, d_wide_row, d_wt_ptr, d_wt_row, d_wt_val, d_minv, d_src_yrow;
};

// GEMM descriptors and task lists of the transforms for one batch size
// (they hold workspace pointers and column counts).  Descriptor
// d = dir * nslots + slot; tasks of all directions are kept in descriptor
// order (d_gtask); the blocked forward and its adjoint have their own
// per-block task lists (d_btask, d_atask).
struct DescTables {
  int64_t B = 0;
  std::vector<GemmDesc> h_gdesc;
  std::vector<GemmTask> h_gtask;
  std::vector<int32_t> h_btask_ptr;   // per block: [fwd, corr, end) offsets into d_btask
  std::vector<int32_t> h_atask_ptr;   // per block: [adjoint apply, adjoint corr, end) offsets into d_atask
  DevBuf d_gdesc, d_gtask, d_btask, d_atask;
  // int8-digit plans: the inverse apply's descriptors and tasks
  std::vector<OzDesc> h_oz;
  std::vector<GemmTask> h_oztask;
  DevBuf d_ozdesc, d_oztask;
  size_t bytes() const {
    return d_gdesc.bytes + d_gtask.bytes + d_btask.bytes + d_atask.bytes + d_ozdesc.bytes + d_oztask.bytes;
  }
};

struct Plan {
  int L = 0, spin = 0;
  uint32_t flags = 0;
  int device = 0;
  int nslots = 0;
  int ncols_per_map = 0;  // 4 (spin 0: +/- x re/im) or 2
  std::vector<int32_t> numer;
  std::string cache_dir;      // placement / tuning cache directory ("" = none)
  std::vector<Slot> slots;
  double max_kappa = 0.0, max_resid = 0.0;
  double fwd_check_err = 0.0;  // plan-time FP64 round trip of one map (see osht_info_t)
  bool fwd_unstable = false;   // spin != 0 and fwd_check_err above the stability bar
  DevBuf d_status;             // OSHT_CHECK_FINITE: int32 set to 1 by a non-finite output
  // device memory
  DevBuf d_cos, d_sin, d_cosh, d_sinh;
  DevBuf d_slots;
  DevBuf d_A, d_Q;            // FP64 blocks (FP32 plans release d_A and keep d_Q for the alias rows)
  DevBuf d_A32, d_Q32;        // FP32 copies, same element offsets (d_Q32 when fp32_fwd)
  bool fp32 = false;          // inverse-side applies on FP32 A_m (OSHT_PREC_FP32, OSHT_PREC_FP32_FWD)
  bool fp32_fwd = false;      // forward coefficient rows on FP32 P_m^{-1} (OSHT_PREC_FP32_FWD, _I8X6, _FWD32)
  int gvar_fwd = 0, gvar_inv = 0;  // stream shapes of the forward and inverse applies (launch_gemm var)
  // inverse apply on int8 digit splits of A_m and X_m (OSHT_PREC_I8X6 / _I8X8):
  // the number of digits, 0 when off; d_A (FP64) stays for the adjoint
  int oz = 0;
  std::vector<int64_t> oz_offA8;  // byte offset of each slot's digit planes in d_A8
  // digit rows are the rings sorted by sin theta (d_ozrow: row -> ring), so
  // that each 64-row tile's negligible Legendre values form one prefix of
  // all-zero 64-deep k-steps; oz_kstart[slot * tiles + tile] is the tile's
  // first k-step with a nonzero digit
  std::vector<int32_t> oz_kstart, oz_rowmap;
  DevBuf d_A8, d_Aexp, d_ozoff, d_ozrow, d_ozkstart;
  // per ring k: every order |m| >= ring_cut[k] has all its Legendre values
  // on ring k below 2^-80, so it adds nothing to ring k's bins in FP64; the
  // fold stops there and the int8 apply leaves out row tiles made only of
  // such rings (built from the FP64 A_m; OSHT_RING_CUT=0 keeps every order)
  std::vector<int32_t> h_ring_cut;
  DevBuf d_ring_cut;
  DevBuf w_X8, w_Xexp;            // per-call digits and exponents of the right-hand sides
  DevBuf d_rings, d_chirp, d_twiddle, d_chirp_tab;
  std::vector<int32_t> h_ring_logM;
  int max_logM = 0;
  // per-call workspace (grown on demand)
  DevBuf w_X, w_Y, w_H, w_T, w_D;
  FwdBlocks fb;
  // descriptor tables per batch size, for the current workspace (at most
  // kMaxTables, least recently used evicted); `tab` is the last call's
  std::vector<std::unique_ptr<DescTables>> tabs;
  DescTables* tab = nullptr;
  static constexpr int kMaxTables = 8;
  int64_t ws_version = 0;     // bumped whenever workspace or descriptor tables are freed
  std::mutex mu;
  Profiler prof;
  int64_t device_bytes() const;
};

// RAII bracket: events around the launches made in its scope.
struct ProfScope {
  Profiler& P;
  const char* name;
  hipStream_t st;
  hipEvent_t e0 = nullptr;
  ProfScope(Profiler& p, const char* n, hipStream_t s) : P(p), name(n), st(s) {
    if (P.wants(n)) {
      e0 = P.get();
      OSHT_HIP(hipEventRecord(e0, st));
    }
  }
  ~ProfScope() {
    if (e0) {
      hipEvent_t e1 = P.get();
      if (hipEventRecord(e1, st) == hipSuccess) P.stat(name).pending.emplace_back(e0, e1);
    }
  }
};

// ---------------------------------------------------------------- launchers
// plan construction (plan.hip)
void build_plan(Plan& p);
// transforms (transform.hip)
// real_maps > 0: the samples f and the coefficients flm are real_maps real
// maps (float64 samples, complex128 coefficients), two per complex map of
// the batch B = ceil(real_maps / 2)
void run_inverse(Plan& p, const double* flm, double* f, int64_t B, hipStream_t st, int64_t real_maps = 0);
void run_forward(Plan& p, const double* f, double* flm, int64_t B, hipStream_t st, int64_t real_maps = 0);
void run_inverse_adjoint(Plan& p, const double* fbar, double* flmbar, int64_t B, hipStream_t st);
void run_forward_adjoint(Plan& p, const double* flmbar, double* fbar, int64_t B, hipStream_t st);
// real maps, spin 0: f real [B][L^2] <-> flm complex [B][L^2] (two maps per
// complex transform)
void run_forward_real(Plan& p, const double* f, double* flm, int64_t B, hipStream_t st);
void run_inverse_real(Plan& p, const double* flm, double* f, int64_t B, hipStream_t st);
// Sizes the workspace and descriptor tables for batch B (synchronous; must
// precede any graph capture of the transforms).
void prepare_transforms(Plan& p, int64_t B);
// Drops every descriptor table (after the device has drained), so that the
// next call rebuilds them: needed when the forward blocks or the plan's
// precision change.
void invalidate_tables(Plan& p);
// OSHT_CHECK_FINITE: scans n doubles for NaN / Inf, setting p.d_status.
void launch_finite_scan(Plan& p, const double* x, int64_t n, hipStream_t st);
// osht_inverse_noalloc (noalloc.hip): the inverse on the library's static
// per-device scratch array; throws OSHT_EINVAL when L and B need more.
void run_inverse_noalloc(Plan& p, const double* flm, double* f, int64_t B, hipStream_t st);
// int8-digit inverse apply (ozaki.hip)
void build_oz_planes(Plan& p);
int oz_x_cols(const Plan& p, int64_t B);   // columns of the right-hand-side digit planes
int oz_x_ld(const Plan& p);                // their leading dimension
void oz_descs(const Plan& p, int64_t B, const double* Y, int8_t* X8, const int32_t* Xexp, std::vector<OzDesc>& descs,
              std::vector<GemmTask>& tasks);
void launch_oz_split_x(const Plan& p, const double* X, int64_t B, int8_t* X8, int32_t* Xexp, hipStream_t st);
void launch_oz_apply(const Plan& p, const OzDesc* d_desc, const GemmTask* d_task, int ntask, hipStream_t st,
                     hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Plan-time FP64 round trip of one map; sets p.fwd_check_err and
// p.fwd_unstable (spin != 0 plans above kSpinForwardStableErr).
constexpr double kSpinForwardStableErr = 1e-8;
// Largest |I - X_m P_m|_max of a usable forward: spin 0 plans above it are
// refused (OSHT_ESINGULAR); spin != 0 plans above it get fwd_unstable.
constexpr double kMaxInvResidual = 1e-10;
void forward_self_check(Plan& p);
// batch scheduler (batch.cpp); jobs validated by the caller
void batch_run(const osht_job_t* jobs, int n, hipStream_t stream, osht_graph_t** graph_inout);

// GEMM (gemm.hip): tasks and descriptors already on the device.
// ApplyInverse32: FP32 A and FP32 B (the inverse apply of FP32 plans).
enum class GemmRole { Plan, ApplyInverse, ApplyInverse32, ApplyForward, Correction, Adjoint };
// With e0/e1, the events take the launch's start and end timestamps.
// var: stream shape of the applies (0 default; 1, 2 alternatives the tuner
// times; all give the same bits).
void launch_gemm(GemmRole role, const GemmDesc* d_desc, const GemmTask* d_task, int ntask, hipStream_t st,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, int var = 0);
constexpr int kGemmVars = 3;
// Builds tasks for descriptors (64 x 64 tiles).
void gemm_tasks(const std::vector<GemmDesc>& descs, std::vector<GemmTask>& tasks);

// ring DFTs (dft.hip)
void build_chirps(Plan& p);
// samples [b][L^2] -> bins [L^2][B] (normalised analysis, scale 1/n_k) or
// unnormalised (scale 1)
void launch_ring_analysis(const Plan& p, const double* f, double* H, int64_t B, bool normalise,
                          hipStream_t st, int64_t real_maps = 0);

// blocked forward sweep (sweep.hip)
void build_fwd_blocks(Plan& p, int b);
// builds the blocks for b; true when the delta solve's LDS need fits
bool fwd_blocks_fit(Plan& p, int b);
// OSHT_TUNE: times the forward for every candidate (b, delta-solve columns
// per group, stream shape of its apply) and the inverse for every stream
// shape of its apply, and keeps the fastest; results cached per (device, L,
// spin, precision) in Plan::cache_dir when set
void autotune(Plan& p);
void run_forward_blocked(Plan& p, const double* f, double* flm, int64_t B, hipStream_t st, int64_t real_maps = 0);
void run_forward_adjoint_blocked(Plan& p, const double* flmbar, double* fbar, int64_t B, hipStream_t st);

// placement (theta.cpp)
int theta_greedy(int L, int32_t* num_out, double* kappa_out);
void theta_alternating(int L, int32_t* num_out);
// the greedy on the current HIP device (throws Error; OSHT_ENOTSUP when
// rocBLAS / rocSOLVER cannot be opened)
void theta_greedy_device(int L, int32_t* num_out, double* kappa_out);
bool theta_greedy_device_available(std::string* why);

constexpr int kTile = 64;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int round_up(int a, int b) { return (int)ceil_div(a, b) * b; }

}  // namespace osht

// Opaque handle of the C ABI.
struct osht_plan {
  osht::Plan p;
};
