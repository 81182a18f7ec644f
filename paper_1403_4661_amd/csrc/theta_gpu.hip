// Greedy colatitude placement (Sec. III-D) on the device: the host greedy's
// algorithm (theta.cpp) with its O(L^4) part on the GPU.
//
// For each order m = L-2 .. 0 (n = L - m):
//   1. rows     R[i * L + t] = Pt[m+i, m](theta_t) for every member t of Theta
//               (one thread per t, the normalised upward recurrence);
//   2. S        S = B^T B, B the n-1 rows of the rings already placed
//               (gathered, then one rocBLAS dgemm);
//   3. T        S = Q T Q^T (rocSOLVER dsytrd), and y = Q^T r for every
//               candidate row r at once (rocSOLVER dormtr applied to R);
//   4. kappa    cond_2([r; B]) of every unused candidate from the secular
//               equation of T + y y^T, one thread per candidate, with the
//               same helpers as the host greedy (secular.hpp);
//   5. choice   the smallest kappa, ties (relative 1e-12) to the smallest
//               numerator, on the host.
// The extreme eigenvalues of T (mu_1, mu_2, mu_n) are bisected on the host
// from T's n diagonal and n-1 off-diagonal entries.
//
// rocBLAS and rocSOLVER are opened with dlopen on first use (by soname, so a
// copy the process has already loaded is reused).
//
// Switched off (kDeviceGreedyEnabled): after the back substitution of the
// secular solve was changed to carry x[i+1], x[i+2] in registers, one run
// left the GPU with a memory fault at L = 5, although the same run's code
// passed every placement test up to L = 1024 before that change, and a CPU
// run of the shared helpers with this layout under AddressSanitizer finds
// no out-of-range access.  Until the cause is shown, the entry point
// reports OSHT_ENOTSUP and plans use the host greedy.

#include <dlfcn.h>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "common.hpp"
#include "host_util.hpp"
#include "secular.hpp"

namespace osht {

namespace {

// R[i * L + t] = Pt[m + i, m](theta_t), i < n = L - m, for all t < L: the
// recurrence of the host rows (seed product, then the three-term upward
// recurrence carried as mantissa * 2^e).
__global__ __launch_bounds__(256) void greedy_rows_kernel(int L, int m, const double* __restrict__ cs,
                                                          const double* __restrict__ sn, double* __restrict__ R) {
#pragma clang fp contract(off)
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L) return;
  const double big = ldexp(1.0, 256), small = ldexp(1.0, -256);
  const double c = cs[t], s = sn[t];
  double p = 0.28209479177387814347;  // 1/sqrt(4 pi)
  int e = 0;
  for (int i = 1; i <= m; ++i) {
    p *= -sqrt((2.0 * i + 1.0) / (2.0 * i)) * s;
    if (p == 0.0) break;
    if (fabs(p) < small) {
      int de;
      p = frexp(p, &de);
      e += de;
    }
  }
  double prev = 0.0, cur = p;
  R[t] = ldexp(cur, e);
  for (int l = m; l < L - 1; ++l) {
    const double den = (double)(l + 1) * (l + 1) - (double)m * m;
    const double a = sqrt((2.0 * l + 1.0) * (2.0 * l + 3.0) / den);
    const double b = (l == m) ? 0.0 : sqrt((2.0 * l + 3.0) * ((double)l * l - (double)m * m) / ((2.0 * l - 1.0) * den));
    const double nxt = a * c * cur - b * prev;
    prev = cur;
    cur = nxt;
    const double mag = fmax(fabs(prev), fabs(cur));
    if (mag > big) {
      prev *= small; cur *= small; e += 256;
    } else if (mag < small && mag > 0.0) {
      prev *= big; cur *= big; e -= 256;
    }
    R[(int64_t)(l + 1 - m) * L + t] = ldexp(cur, e);
  }
}

// B, column-major (n-1) x n: B[j + i (n-1)] = R[i L + tsel[m+1+j]], the row of
// the ring k = m+1+j (placed at member tsel[k]).
__global__ __launch_bounds__(256) void greedy_gather_kernel(int L, int m, int n, const int32_t* __restrict__ tsel,
                                                            const double* __restrict__ R, double* __restrict__ B) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nb = (int64_t)(n - 1) * n;
  if (e >= nb) return;
  const int j = (int)(e % (n - 1)), i = (int)(e / (n - 1));
  B[e] = R[(int64_t)i * L + tsel[m + 1 + j]];
}

// kap[c] = cond_2([r; B]) for candidate c (member cand[c]); Y[i L + t] is
// y = Q^T r of member t.  T (diagonal D, off-diagonal E) is staged in LDS;
// the 4n work entries of candidate c sit at work[k * nc + c].
__global__ __launch_bounds__(64) void greedy_secular_kernel(int n, int L, int nc, const int32_t* __restrict__ cand,
                                                           const double* __restrict__ D, const double* __restrict__ E,
                                                           const double* __restrict__ Y, double mu1, double mu2,
                                                           double mun, double* __restrict__ work,
                                                           double* __restrict__ kap) {
#pragma clang fp contract(off)
  extern __shared__ double tri[];  // D then E
  for (int i = threadIdx.x; i < n; i += blockDim.x) tri[i] = D[i];
  for (int i = threadIdx.x; i < n - 1; i += blockDim.x) tri[n + i] = E[i];
  __syncthreads();
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const secular::View<const double> y{Y + cand[c], L};
  double rr = 0.0;
  for (int i = 0; i < n; ++i) rr += y[i] * y[i];
  kap[c] = secular::candidate_kappa(n, tri, tri + n, y, rr, mu1, mu2, mun, secular::View<double>{work + c, nc});
}

// rocBLAS / rocSOLVER entry points used here
struct Solver {
  bool ok = false;
  std::string why;
  decltype(&rocblas_create_handle) create = nullptr;
  decltype(&rocblas_destroy_handle) destroy = nullptr;
  decltype(&rocblas_set_stream) set_stream = nullptr;
  decltype(&rocblas_dgemm) dgemm = nullptr;
  decltype(&rocsolver_dsytrd) sytrd = nullptr;
  decltype(&rocsolver_dormtr) ormtr = nullptr;
};

void* open_first(std::initializer_list<const char*> names) {
  for (const char* n : names)
    if (void* h = dlopen(n, RTLD_NOW | RTLD_LOCAL)) return h;
  return nullptr;
}

const Solver& solver() {
  static const Solver s = [] {
    Solver r;
    void* hb = open_first({"librocblas.so.5", "librocblas.so"});
    void* hs = open_first({"librocsolver.so.0", "librocsolver.so"});
    if (!hb || !hs) {
      r.why = std::string("dlopen: ") + (dlerror() ? dlerror() : "library not found");
      return r;
    }
    r.create = reinterpret_cast<decltype(r.create)>(dlsym(hb, "rocblas_create_handle"));
    r.destroy = reinterpret_cast<decltype(r.destroy)>(dlsym(hb, "rocblas_destroy_handle"));
    r.set_stream = reinterpret_cast<decltype(r.set_stream)>(dlsym(hb, "rocblas_set_stream"));
    r.dgemm = reinterpret_cast<decltype(r.dgemm)>(dlsym(hb, "rocblas_dgemm"));
    r.sytrd = reinterpret_cast<decltype(r.sytrd)>(dlsym(hs, "rocsolver_dsytrd"));
    r.ormtr = reinterpret_cast<decltype(r.ormtr)>(dlsym(hs, "rocsolver_dormtr"));
    r.ok = r.create && r.destroy && r.set_stream && r.dgemm && r.sytrd && r.ormtr;
    if (!r.ok) r.why = "a rocBLAS / rocSOLVER entry point is missing";
    return r;
  }();
  return s;
}

void check_rb(rocblas_status st, const char* what) {
  if (st != rocblas_status_success)
    throw Error{OSHT_EHIP, std::string(what) + " failed (rocblas_status " + std::to_string((int)st) + ")"};
}

}  // namespace

constexpr bool kDeviceGreedyEnabled = false;

bool theta_greedy_device_available(std::string* why) {
  if (!kDeviceGreedyEnabled) {
    if (why) *why = "switched off";
    return false;
  }
  const Solver& s = solver();
  if (!s.ok && why) *why = s.why;
  return s.ok;
}

void theta_greedy_device(int L, int32_t* num_out, double* kappa_out) {
  if (!kDeviceGreedyEnabled)
    throw Error{OSHT_ENOTSUP, "the device greedy is switched off (an unexplained GPU memory fault); use the host greedy"};
  const Solver& sv = solver();
  if (!sv.ok) throw Error{OSHT_ENOTSUP, "device placement needs rocBLAS and rocSOLVER: " + sv.why};
  std::vector<int32_t> chosen(L, 0);  // numerator of ring k
  std::vector<char> used(L, 0);
  std::vector<double> cs(L), sn(L);
  for (int t = 0; t < L; ++t) ring_trig(L, 2 * t + 1, &cs[t], &sn[t], nullptr, nullptr);
  chosen[L - 1] = 2 * ((L - 1) / 2) + 1;
  used[(chosen[L - 1] - 1) / 2] = 1;
  if (kappa_out) kappa_out[L - 1] = 1.0;
  if (L == 1) {
    num_out[0] = chosen[0];
    return;
  }
  const size_t LL = (size_t)L * L;
  DevBuf d_cs, d_sn, d_R, d_B, d_S, d_D, d_E, d_tau, d_tsel, d_cand, d_kap, d_work;
  upload(d_cs, cs);
  upload(d_sn, sn);
  d_R.alloc(sizeof(double) * LL);
  d_B.alloc(sizeof(double) * LL);
  d_S.alloc(sizeof(double) * LL);
  d_D.alloc(sizeof(double) * L);
  d_E.alloc(sizeof(double) * L);
  d_tau.alloc(sizeof(double) * L);
  d_cand.alloc(sizeof(int32_t) * L);
  d_kap.alloc(sizeof(double) * L);
  d_work.alloc(sizeof(double) * 4 * LL);
  std::vector<int32_t> tsel(L, 0);  // member placed at ring k (k > m)
  tsel[L - 1] = (chosen[L - 1] - 1) / 2;
  upload(d_tsel, tsel);
  rocblas_handle h = nullptr;
  check_rb(sv.create(&h), "rocblas_create_handle");
  struct HandleGuard {
    const Solver& sv;
    rocblas_handle h;
    ~HandleGuard() { sv.destroy(h); }
  } guard{sv, h};
  check_rb(sv.set_stream(h, nullptr), "rocblas_set_stream");
  std::vector<double> hD(L), hE(L), hkap(L);
  std::vector<int32_t> cand;
  const double one = 1.0, zero = 0.0;
  for (int m = L - 2; m >= 0; --m) {
    const int n = L - m;
    hipLaunchKernelGGL(greedy_rows_kernel, dim3((unsigned)ceil_div(L, 256)), dim3(256), 0, nullptr, L, m,
                       d_cs.as<double>(), d_sn.as<double>(), d_R.as<double>());
    OSHT_HIP(hipGetLastError());
    hipLaunchKernelGGL(greedy_gather_kernel, dim3((unsigned)ceil_div((int64_t)(n - 1) * n, 256)), dim3(256), 0, nullptr,
                       L, m, n, d_tsel.as<int32_t>(), d_R.as<double>(), d_B.as<double>());
    OSHT_HIP(hipGetLastError());
    check_rb(sv.dgemm(h, rocblas_operation_transpose, rocblas_operation_none, n, n, n - 1, &one, d_B.as<double>(),
                      n - 1, d_B.as<double>(), n - 1, &zero, d_S.as<double>(), n),
             "rocblas_dgemm");
    check_rb(sv.sytrd(h, rocblas_fill_lower, n, d_S.as<double>(), n, d_D.as<double>(), d_E.as<double>(),
                      d_tau.as<double>()),
             "rocsolver_dsytrd");
    // R <- R Q: row t of R becomes (Q^T r_t)^T
    check_rb(sv.ormtr(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_none, L, n, d_S.as<double>(), n,
                      d_tau.as<double>(), d_R.as<double>(), L),
             "rocsolver_dormtr");
    OSHT_HIP(hipMemcpy(hD.data(), d_D.p, sizeof(double) * n, hipMemcpyDeviceToHost));
    OSHT_HIP(hipMemcpy(hE.data(), d_E.p, sizeof(double) * (n - 1), hipMemcpyDeviceToHost));
    const double mu1 = secular::tri_eig(n, hD.data(), hE.data(), 0);
    const double mu2 = secular::tri_eig(n, hD.data(), hE.data(), 1);
    const double mun = secular::tri_eig(n, hD.data(), hE.data(), n - 1);
    cand.clear();
    for (int t = 0; t < L; ++t)
      if (!used[t]) cand.push_back(t);
    const int nc = (int)cand.size();
    OSHT_HIP(hipMemcpy(d_cand.p, cand.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(greedy_secular_kernel, dim3((unsigned)ceil_div(nc, 64)), dim3(64),
                       sizeof(double) * (2 * (size_t)n), nullptr, n, L, nc, d_cand.as<int32_t>(), d_D.as<double>(),
                       d_E.as<double>(), d_R.as<double>(), mu1, mu2, mun, d_work.as<double>(), d_kap.as<double>());
    OSHT_HIP(hipGetLastError());
    OSHT_HIP(hipMemcpy(hkap.data(), d_kap.p, sizeof(double) * nc, hipMemcpyDeviceToHost));
    double kmin = std::numeric_limits<double>::infinity();
    for (int c = 0; c < nc; ++c) kmin = std::min(kmin, hkap[c]);
    int pick = 0;
    for (int c = 0; c < nc; ++c)
      if (hkap[c] <= kmin * (1.0 + 1e-12)) {
        pick = c;
        break;
      }
    chosen[m] = 2 * cand[pick] + 1;
    used[cand[pick]] = 1;
    tsel[m] = cand[pick];
    if (kappa_out) kappa_out[m] = hkap[pick];
    OSHT_HIP(hipMemcpy(d_tsel.as<int32_t>() + m, &tsel[m], sizeof(int32_t), hipMemcpyHostToDevice));
  }
  for (int k = 0; k < L; ++k) num_out[k] = chosen[k];
}

}  // namespace osht
