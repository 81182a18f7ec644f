// extern "C" entry points of libosht (declared in include/osht.h).

#include <unistd.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>

#include "common.hpp"
#include "host_util.hpp"

using osht::Error;
using osht::Plan;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

bool valid_permutation(int L, const std::vector<int32_t>& num) {
  if ((int)num.size() != L) return false;
  std::vector<char> seen(L, 0);
  for (int32_t n : num) {
    if (n < 1 || n > 2 * L - 1 || (n % 2) == 0) return false;
    if (seen[(n - 1) / 2]) return false;
    seen[(n - 1) / 2] = 1;
  }
  return true;
}

std::string cache_path(const char* dir, int L) {
  return std::string(dir) + "/theta_greedy_L" + std::to_string(L) + ".txt";
}

// 1: read ok, 0: no file, -1: malformed
int read_cache(const std::string& path, int L, std::vector<int32_t>& num) {
  std::ifstream in(path);
  if (!in) return 0;
  num.clear();
  std::string line;
  while (std::getline(in, line)) {
    size_t a = line.find_first_not_of(" \t\r");
    if (a == std::string::npos || line[a] == '#') continue;
    char* end = nullptr;
    long v = std::strtol(line.c_str() + a, &end, 10);
    if (end == line.c_str() + a) return -1;
    num.push_back((int32_t)v);
  }
  return valid_permutation(L, num) ? 1 : -1;
}

void write_cache(const std::string& path, const std::vector<int32_t>& num, const std::vector<double>& kap) {
  std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  std::ofstream out(tmp);
  if (!out) return;
  for (int32_t n : num) out << n << "\n";
  double km = 0.0;
  for (double k : kap) km = std::max(km, k);
  char buf[64];
  std::snprintf(buf, sizeof buf, "# max_kappa %.6e\n", km);
  out << buf;
  out.close();
  if (out) std::rename(tmp.c_str(), path.c_str());
  else std::remove(tmp.c_str());
}

bool overlaps(const void* a, const void* b, size_t bytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Forward-direction calls on a plan whose forward failed the plan-time
// self-check (spin != 0 only) are refused unless the plan forces them.
bool forward_refused(const Plan& p) { return p.fwd_unstable && !(p.flags & OSHT_SPIN_FWD_FORCE); }

std::string refused_message(const Plan& p) {
  char buf[256];
  std::snprintf(buf, sizeof buf,
                "the spin %d forward is unstable on this plan at L = %d (plan-time round trip error %.3g); "
                "create the plan with OSHT_SPIN_FWD_FORCE to run it anyway",
                p.spin, p.L, p.fwd_check_err);
  return buf;
}

template <class Fn>
int run_transform(const osht_plan_t* plan, const void* in, void* out, int64_t batch, hipStream_t stream,
                  bool forward_dir, Fn fn) {
  if (!plan) return fail(OSHT_EINVAL, "plan is NULL");
  if (!in || !out) return fail(OSHT_EINVAL, "input or output pointer is NULL");
  if (batch < 1 || batch > 65535) return fail(OSHT_EINVAL, "batch must be in [1, 65535]");
  Plan& p = const_cast<osht_plan_t*>(plan)->p;
  const size_t bytes = sizeof(double) * 2 * (size_t)p.L * p.L * (size_t)batch;
  if (overlaps(in, out, bytes)) return fail(OSHT_EINVAL, "input and output buffers overlap");
  if (forward_dir && forward_refused(p)) return fail(OSHT_ENOTSUP, refused_message(p));
  try {
    std::lock_guard<std::mutex> lk(p.mu);
    DeviceGuard g(p.device);
    fn(p, static_cast<const double*>(in), static_cast<double*>(out));
    if (p.flags & OSHT_CHECK_FINITE)
      osht::launch_finite_scan(p, static_cast<const double*>(out), (int64_t)(bytes / sizeof(double)), stream);
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(OSHT_ENOMEM, "host allocation failed");
  }
  return OSHT_OK;
}

// As run_transform, with one side real (float64) and the other complex128.
template <class Fn>
int run_real_transform(const osht_plan_t* plan, const void* in, int64_t bin, bool in_cplx, void* out, int64_t bout,
                       bool out_cplx, hipStream_t stream, Fn fn) {
  if (!plan) return fail(OSHT_EINVAL, "plan is NULL");
  if (!in || !out) return fail(OSHT_EINVAL, "input or output pointer is NULL");
  if (bin < 1 || bin > 65535) return fail(OSHT_EINVAL, "batch must be in [1, 65535]");
  Plan& p = const_cast<osht_plan_t*>(plan)->p;
  if (p.spin != 0) return fail(OSHT_ENOTSUP, "real-map transforms are defined for spin 0 only");
  const size_t n = (size_t)p.L * p.L;
  const size_t ib = sizeof(double) * n * (size_t)bin * (in_cplx ? 2 : 1);
  const size_t ob = sizeof(double) * n * (size_t)bout * (out_cplx ? 2 : 1);
  const char* x = static_cast<const char*>(in);
  const char* y = static_cast<const char*>(out);
  if (x < y + ob && y < x + ib) return fail(OSHT_EINVAL, "input and output buffers overlap");
  try {
    std::lock_guard<std::mutex> lk(p.mu);
    DeviceGuard g(p.device);
    fn(p, static_cast<const double*>(in), static_cast<double*>(out));
    if (p.flags & OSHT_CHECK_FINITE)
      osht::launch_finite_scan(p, static_cast<const double*>(out), (int64_t)(ob / sizeof(double)), stream);
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(OSHT_ENOMEM, "host allocation failed");
  }
  return OSHT_OK;
}

}  // namespace

extern "C" {

const char* osht_strerror(int code) {
  switch (code) {
    case OSHT_OK: return "success";
    case OSHT_EINVAL: return "invalid argument";
    case OSHT_ENOMEM: return "out of memory";
    case OSHT_EHIP: return "HIP runtime error";
    case OSHT_ESINGULAR: return "a per-order system failed its inversion check";
    case OSHT_ENOTSUP: return "not supported by this plan (flags or an unstable spin forward)";
    case OSHT_EIO: return "placement cache file unreadable or malformed";
    case OSHT_ENONFINITE: return "a transform output held NaN or Inf";
    default: return "unknown error";
  }
}

const char* osht_last_error_message(void) { return g_last_error.c_str(); }

int osht_theta_greedy(int L, int32_t* numerators_out, double* kappa_out) {
  if (L < 1 || L > 4096 || !numerators_out) return fail(OSHT_EINVAL, "L must be in [1, 4096] and the output non-NULL");
  try {
    osht::theta_greedy(L, numerators_out, kappa_out);
  } catch (const std::bad_alloc&) {
    return fail(OSHT_ENOMEM, "host allocation failed");
  }
  return OSHT_OK;
}

int osht_theta_greedy_device(int L, int32_t* numerators_out, double* kappa_out) {
  if (L < 1 || L > 4096 || !numerators_out) return fail(OSHT_EINVAL, "L must be in [1, 4096] and the output non-NULL");
  try {
    osht::theta_greedy_device(L, numerators_out, kappa_out);
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(OSHT_ENOMEM, "host allocation failed");
  }
  return OSHT_OK;
}

int osht_theta_alternating(int L, int32_t* numerators_out) {
  if (L < 1 || L > 4096 || !numerators_out) return fail(OSHT_EINVAL, "L must be in [1, 4096] and the output non-NULL");
  osht::theta_alternating(L, numerators_out);
  return OSHT_OK;
}

int osht_plan_create(int L, int spin, uint32_t flags, const char* theta_cache_dir, osht_plan_t** out) {
  if (!out) return fail(OSHT_EINVAL, "out is NULL");
  *out = nullptr;
  if (L < 1 || L > 4096) return fail(OSHT_EINVAL, "L must be in [1, 4096]");
  if (spin <= -L || spin >= L) return fail(OSHT_EINVAL, "|spin| must be < L");
  const uint32_t prec = flags & OSHT_PREC_MASK, theta = flags & OSHT_THETA_MASK;
  if (prec != OSHT_PREC_FP64 && prec != OSHT_PREC_FP32 && prec != OSHT_PREC_FP32_FWD && prec != OSHT_PREC_I8X6 &&
      prec != OSHT_PREC_I8X8 && prec != OSHT_PREC_FWD32)
    return fail(OSHT_ENOTSUP, "precision must be OSHT_PREC_FP64, _FP32, _FP32_FWD, _I8X6, _I8X8 or _FWD32");
  if (theta != OSHT_THETA_GREEDY && theta != OSHT_THETA_ALTERNATING) return fail(OSHT_EINVAL, "unknown placement flag");
  if (flags & ~(OSHT_PREC_MASK | OSHT_THETA_MASK | OSHT_TUNE | OSHT_SPIN_FWD_FORCE | OSHT_CHECK_FINITE))
    return fail(OSHT_EINVAL, "unknown flag bits");
  osht_plan_t* h = nullptr;
  try {
    h = new osht_plan_t;
    Plan& p = h->p;
    p.L = L;
    p.spin = spin;
    p.flags = flags;
    p.fp32 = prec == OSHT_PREC_FP32 || prec == OSHT_PREC_FP32_FWD;
    p.fp32_fwd = prec == OSHT_PREC_FP32_FWD || prec == OSHT_PREC_I8X6 || prec == OSHT_PREC_FWD32;
    p.oz = prec == OSHT_PREC_I8X6 ? 6 : prec == OSHT_PREC_I8X8 ? 8 : 0;
    if (theta_cache_dir) p.cache_dir = theta_cache_dir;
    OSHT_HIP(hipGetDevice(&p.device));
    p.numer.assign(L, 0);
    if (theta == OSHT_THETA_ALTERNATING) {
      osht::theta_alternating(L, p.numer.data());
    } else {
      int got = 0;
      if (theta_cache_dir) {
        got = read_cache(cache_path(theta_cache_dir, L), L, p.numer);
        if (got < 0) throw Error{OSHT_EIO, "malformed placement cache " + cache_path(theta_cache_dir, L)};
      }
      if (got == 0) {
        std::vector<double> kap(L);
        p.numer.assign(L, 0);
        if (osht::theta_greedy_device_available(nullptr)) osht::theta_greedy_device(L, p.numer.data(), kap.data());
        else osht::theta_greedy(L, p.numer.data(), kap.data());
        if (theta_cache_dir) write_cache(cache_path(theta_cache_dir, L), p.numer, kap);
      }
    }
    osht::build_plan(p);
  } catch (const Error& e) {
    delete h;
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    delete h;
    return fail(OSHT_ENOMEM, "host allocation failed");
  }
  *out = h;
  return OSHT_OK;
}

int osht_plan_destroy(osht_plan_t* plan) {
  if (!plan) return OSHT_OK;
  {
    DeviceGuard g(plan->p.device);
    (void)hipDeviceSynchronize();
    delete plan;
  }
  return OSHT_OK;
}

int osht_plan_info(const osht_plan_t* plan, osht_info_t* out) {
  if (!plan || !out) return fail(OSHT_EINVAL, "NULL argument");
  const Plan& p = plan->p;
  std::memset(out, 0, sizeof *out);
  out->L = p.L;
  out->spin = p.spin;
  out->flags = p.flags;
  out->nsamples = (int64_t)p.L * p.L;
  out->ncoeffs = (int64_t)p.L * p.L;
  out->device_bytes = p.device_bytes();
  out->max_kappa = p.max_kappa;
  out->max_inv_residual = p.max_resid;
  out->fwd_check_err = p.fwd_check_err;
  out->fwd_unstable = p.fwd_unstable ? 1 : 0;
  return OSHT_OK;
}

int osht_plan_theta(const osht_plan_t* plan, int32_t* numerators_host) {
  if (!plan || !numerators_host) return fail(OSHT_EINVAL, "NULL argument");
  std::memcpy(numerators_host, plan->p.numer.data(), sizeof(int32_t) * plan->p.L);
  return OSHT_OK;
}

int osht_inverse(const osht_plan_t* plan, const void* flm, void* f, int64_t batch, hipStream_t stream) {
  return run_transform(plan, flm, f, batch, stream, false,
                       [&](Plan& p, const double* a, double* b) { osht::run_inverse(p, a, b, batch, stream); });
}

int osht_inverse_noalloc(const osht_plan_t* plan, const void* flm, void* f, int64_t batch, hipStream_t stream) {
  return run_transform(plan, flm, f, batch, stream, false,
                       [&](Plan& p, const double* a, double* b) { osht::run_inverse_noalloc(p, a, b, batch, stream); });
}

int osht_forward(const osht_plan_t* plan, const void* f, void* flm, int64_t batch, hipStream_t stream) {
  return run_transform(plan, f, flm, batch, stream, true,
                       [&](Plan& p, const double* a, double* b) { osht::run_forward(p, a, b, batch, stream); });
}

int osht_forward_real(const osht_plan_t* plan, const void* f, void* flm, int64_t batch, hipStream_t stream) {
  return run_real_transform(plan, f, batch, false, flm, batch, true, stream,
                            [&](Plan& p, const double* a, double* b) { osht::run_forward_real(p, a, b, batch, stream); });
}

int osht_inverse_real(const osht_plan_t* plan, const void* flm, void* f, int64_t batch, hipStream_t stream) {
  return run_real_transform(plan, flm, batch, true, f, batch, false, stream,
                            [&](Plan& p, const double* a, double* b) { osht::run_inverse_real(p, a, b, batch, stream); });
}

int osht_inverse_adjoint(const osht_plan_t* plan, const void* f_bar, void* flm_bar, int64_t batch, hipStream_t stream) {
  return run_transform(plan, f_bar, flm_bar, batch, stream, false,
                       [&](Plan& p, const double* a, double* b) { osht::run_inverse_adjoint(p, a, b, batch, stream); });
}

int osht_forward_adjoint(const osht_plan_t* plan, const void* flm_bar, void* f_bar, int64_t batch, hipStream_t stream) {
  return run_transform(plan, flm_bar, f_bar, batch, stream, true,
                       [&](Plan& p, const double* a, double* b) { osht::run_forward_adjoint(p, a, b, batch, stream); });
}

int osht_plan_set_profiling(osht_plan_t* plan, int enable, const char* only_name) {
  if (!plan) return fail(OSHT_EINVAL, "plan is NULL");
  Plan& p = plan->p;
  try {
    std::lock_guard<std::mutex> lk(p.mu);
    DeviceGuard g(p.device);
    p.prof.reset();
    p.prof.enabled = enable != 0;
    p.prof.only = only_name ? only_name : "";
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  }
  return OSHT_OK;
}

int osht_plan_kernel_time(osht_plan_t* plan, const char* name, int64_t* launches, double* total_ms) {
  if (!plan || !name || !launches || !total_ms) return fail(OSHT_EINVAL, "NULL argument");
  Plan& p = plan->p;
  try {
    std::lock_guard<std::mutex> lk(p.mu);
    DeviceGuard g(p.device);
    *launches = 0;
    *total_ms = 0.0;
    for (auto& kv : p.prof.stats) {
      if (kv.first == name) {
        p.prof.flush(kv.second);
        *launches = kv.second.count;
        *total_ms = kv.second.ms;
      }
    }
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  }
  return OSHT_OK;
}

int osht_plan_status(osht_plan_t* plan, int32_t* status) {
  if (!plan || !status) return fail(OSHT_EINVAL, "NULL argument");
  Plan& p = plan->p;
  *status = OSHT_OK;
  if (!(p.flags & OSHT_CHECK_FINITE)) return OSHT_OK;
  try {
    std::lock_guard<std::mutex> lk(p.mu);
    DeviceGuard g(p.device);
    OSHT_HIP(hipDeviceSynchronize());
    int32_t v = 0;
    const int32_t zero = 0;
    OSHT_HIP(hipMemcpy(&v, p.d_status.p, sizeof v, hipMemcpyDeviceToHost));
    OSHT_HIP(hipMemcpy(p.d_status.p, &zero, sizeof zero, hipMemcpyHostToDevice));
    if (v) *status = OSHT_ENONFINITE;
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  }
  return OSHT_OK;
}

int osht_batch_run(const osht_job_t* jobs, int njobs, hipStream_t stream, osht_graph_t** graph_inout) {
  if (njobs < 0 || (njobs > 0 && !jobs)) return fail(OSHT_EINVAL, "bad job list");
  for (int i = 0; i < njobs; ++i) {
    const osht_job_t& j = jobs[i];
    if (!j.plan || !j.in || !j.out) return fail(OSHT_EINVAL, "job " + std::to_string(i) + ": NULL plan or buffer");
    if (j.direction < OSHT_DIR_INVERSE || j.direction > OSHT_DIR_FORWARD_ADJOINT || j.reserved != 0)
      return fail(OSHT_EINVAL, "job " + std::to_string(i) + ": bad direction");
    if (j.batch < 1 || j.batch > 65535) return fail(OSHT_EINVAL, "job " + std::to_string(i) + ": batch out of range");
    const size_t bytes = sizeof(double) * 2 * (size_t)j.plan->p.L * j.plan->p.L * (size_t)j.batch;
    if (overlaps(j.in, j.out, bytes)) return fail(OSHT_EINVAL, "job " + std::to_string(i) + ": in and out overlap");
    for (int k = 0; k < i; ++k)
      if (jobs[k].plan == j.plan && jobs[k].batch != j.batch)
        return fail(OSHT_EINVAL, "jobs of one plan must share the batch size");
    if ((j.direction == OSHT_DIR_FORWARD || j.direction == OSHT_DIR_FORWARD_ADJOINT) && forward_refused(j.plan->p))
      return fail(OSHT_ENOTSUP, "job " + std::to_string(i) + ": " + refused_message(j.plan->p));
  }
  if (njobs == 0) return OSHT_OK;
  try {
    osht::batch_run(jobs, njobs, stream, graph_inout);
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(OSHT_ENOMEM, "host allocation failed");
  }
  return OSHT_OK;
}

}  // extern "C"
