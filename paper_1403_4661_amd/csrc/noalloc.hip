// Inverse SHT that allocates no device memory (osht_inverse_noalloc).
//
// The per-call workspace of the inverse -- the GEMM descriptor and task
// tables, the slot-layout coefficients X, the per-order outputs Y and the
// ring bins H -- lives in one file-scope device array, `scratch`, of
// kScratchBytes, instead of the plan's workspace.  Every GPU the library
// runs on holds its own copy until the process ends; its device address is
// taken once per device with hipGetSymbolAddress and only that address is
// passed to kernels.  The descriptor and task tables are written on the
// device by a small kernel (no host copies).  The kernels are the ones of
// osht_inverse (coefficient transpose, order-wise apply, fold, ring
// synthesis), so the results are identical.
//
// Calls on one GPU share its array: calls that overlap in time on one GPU
// race.  Nothing in the array needs to start at zero (every byte a call
// reads was written earlier in the same call).

#include <mutex>

#include "xform.hpp"

namespace osht {

void launch_fold(const Plan& p, const double* Y, double* H, int64_t B, hipStream_t st);
void launch_ring_synthesis(const Plan& p, const double* H, int scale_inv_n, double* f, int64_t B, hipStream_t st,
                           int64_t real_maps);
void launch_coef_to_slots(const Plan& p, const double* flm, double* X, int64_t B, hipStream_t st, bool f32,
                          int64_t real_maps);

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (the device must be current).
void* scratch_ptr(int dev) {
  OSHT_CHECK(dev >= 0 && dev < kMaxDevices, OSHT_ENOTSUP, "device index out of range for the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    OSHT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    OSHT_CHECK(ptr != nullptr, OSHT_EHIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

struct Layout {
  size_t desc, task, X, Y, H, end;
  int ntask, mt, nt;
};

Layout layout(const Plan& p, int64_t B) {
  Layout l{};
  const int64_t ncols = p.ncols_per_map * B;
  l.mt = (int)ceil_div(p.L, kTile);
  l.nt = (int)ceil_div(ncols, kTile);
  l.ntask = p.nslots * l.mt * l.nt;
  size_t off = 0;
  l.desc = off;
  off = align256(off + sizeof(GemmDesc) * (size_t)p.nslots);
  l.task = off;
  off = align256(off + sizeof(GemmTask) * (size_t)l.ntask);
  const size_t xy = sizeof(double) * (size_t)p.nslots * p.L * ncols;
  l.X = off;
  off = align256(off + xy);
  l.Y = off;
  off = align256(off + xy);
  l.H = off;
  off = align256(off + sizeof(double) * 2 * (size_t)p.L * p.L * B);
  l.end = off;
  return l;
}

// The inverse apply's descriptors (one per slot, as the plan's own tables
// hold them, with X and Y in scratch) and its tasks in descriptor order.
__global__ __launch_bounds__(256) void inverse_tables_kernel(const Slot* __restrict__ slots, int nslots, int L,
                                                             int ncols, const void* __restrict__ A, int f32,
                                                             unsigned char* __restrict__ base, Layout l) {
  GemmDesc* desc = reinterpret_cast<GemmDesc*>(base + l.desc);
  GemmTask* task = reinterpret_cast<GemmTask*>(base + l.task);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nslots; i += stride) {
    const Slot sl = slots[i];
    GemmDesc d{};
    const int64_t o = i * (int64_t)L * ncols;
    if (f32) {
      d.A = static_cast<const float*>(A) + sl.offA;
      d.fp32 = 1;
      d.B = reinterpret_cast<const double*>(reinterpret_cast<const float*>(base + l.X) + o);
      d.C = reinterpret_cast<double*>(reinterpret_cast<float*>(base + l.Y) + o);
      d.b32 = 1;
      d.c32 = 1;
    } else {
      d.A = static_cast<const double*>(A) + sl.offA;
      d.B = reinterpret_cast<const double*>(base + l.X) + o;
      d.C = reinterpret_cast<double*>(base + l.Y) + o;
    }
    d.sAr = 1;
    d.sAc = sl.ldA;
    d.sBr = ncols;
    d.sBc = 1;
    d.sCr = ncols;
    d.sCc = 1;
    d.M = L;
    d.N = ncols;
    d.K = sl.K;
    d.alpha = 1.0;
    d.beta = 0.0;
    desc[i] = d;
  }
  const int per = l.mt * l.nt;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < l.ntask; t += stride) {
    const int i = (int)(t / per), r = (int)(t - (int64_t)i * per);
    task[t] = GemmTask{i, r / l.nt, r % l.nt, 0};
  }
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

size_t noalloc_inverse_need(const Plan& p, int64_t B) { return layout(p, B).end; }

void run_inverse_noalloc(Plan& p, const double* flm, double* f, int64_t B, hipStream_t st) {
  OSHT_CHECK(p.oz == 0, OSHT_ENOTSUP, "osht_inverse_noalloc: not available on int8-digit (I8X6 / I8X8) plans");
  const Layout l = layout(p, B);
  OSHT_CHECK(l.end <= kScratchBytes, OSHT_EINVAL,
             "osht_inverse_noalloc: L = " + std::to_string(p.L) + ", batch " + std::to_string(B) + " needs " +
                 std::to_string(l.end) + " bytes of scratch, more than its " + std::to_string(kScratchBytes));
  unsigned char* base = static_cast<unsigned char*>(scratch_ptr(p.device));
  const int64_t ncols = p.ncols_per_map * B;
  const void* A = p.fp32 ? static_cast<const void*>(p.d_A32.p) : static_cast<const void*>(p.d_A.p);
  const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(std::max<int64_t>(l.ntask, p.nslots), 256), 1024);
  hipLaunchKernelGGL(inverse_tables_kernel, dim3(blocks), dim3(256), 0, st, p.d_slots.as<Slot>(), p.nslots, p.L,
                     (int)ncols, A, p.fp32 ? 1 : 0, base, l);
  OSHT_HIP(hipGetLastError());
  double* X = reinterpret_cast<double*>(base + l.X);
  double* Y = reinterpret_cast<double*>(base + l.Y);
  double* H = reinterpret_cast<double*>(base + l.H);
  launch_coef_to_slots(p, flm, X, B, st, p.fp32, 0);
  launch_gemm(p.fp32 ? GemmRole::ApplyInverse32 : GemmRole::ApplyInverse,
              reinterpret_cast<const GemmDesc*>(base + l.desc), reinterpret_cast<const GemmTask*>(base + l.task),
              l.ntask, st, nullptr, nullptr, p.gvar_inv);
  launch_fold(p, Y, H, B, st);
  launch_ring_synthesis(p, H, 0, f, B, st, 0);
}

}  // namespace osht
