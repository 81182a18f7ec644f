// Host-side helpers shared by the plan builder and the placement greedy.
#pragma once

#include <algorithm>
#include <condition_variable>
#include <mutex>
#include <cmath>
#include <cstdint>
#include <functional>
#include <thread>
#include <vector>

namespace osht {

// Number of worker threads for host loops (hardware concurrency, at least 1,
// at most 16).
inline int host_threads() {
  unsigned n = std::thread::hardware_concurrency();
  if (n == 0) n = 1;
  return (int)std::min(n, 16u);
}

// Persistent pool of host worker threads.  parallel_for(begin, end, fn)
// runs fn(i) for every i in [begin, end), split in contiguous chunks over the
// workers and the calling thread; small ranges run inline.  Calls are
// serialised by a mutex (one parallel region at a time).
class HostPool {
 public:
  static HostPool& get() {
    static HostPool pool(host_threads());
    return pool;
  }
  void run(int64_t begin, int64_t end, const std::function<void(int64_t)>& fn, int64_t min_per_thread) {
    int64_t n = end - begin;
    if (n <= 0) return;
    int nt = (int)std::min<int64_t>(nworkers_ + 1, std::max<int64_t>(1, n / std::max<int64_t>(1, min_per_thread)));
    if (nt <= 1 || in_region()) {  // nested regions run inline
      for (int64_t i = begin; i < end; ++i) fn(i);
      return;
    }
    std::lock_guard<std::mutex> region(region_);
    in_region() = true;
    struct Reset { ~Reset() { in_region() = false; } } reset;
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn; begin_ = begin; n_ = n; nt_ = nt; pending_ = nt - 1; ++gen_;
    }
    cv_.notify_all();
    chunk(0);
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return pending_ == 0; });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true; ++gen_;
    }
    cv_.notify_all();
    for (auto& t : threads_) t.join();
  }

 private:
  explicit HostPool(int nthreads) : nworkers_(std::max(0, nthreads - 1)) {
    for (int w = 0; w < nworkers_; ++w) threads_.emplace_back([this, w] { loop(w + 1); });
  }
  static bool& in_region() {
    static thread_local bool flag = false;
    return flag;
  }
  void chunk(int t) {
    int64_t lo = begin_ + n_ * t / nt_, hi = begin_ + n_ * (t + 1) / nt_;
    for (int64_t i = lo; i < hi; ++i) (*fn_)(i);
  }
  void loop(int id) {
    uint64_t seen = 0;
    for (;;) {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
      if (stop_) return;
      seen = gen_;
      if (id >= nt_) continue;
      lk.unlock();
      in_region() = true;
      chunk(id);
      in_region() = false;
      lk.lock();
      if (--pending_ == 0) done_.notify_one();
    }
  }
  int nworkers_;
  std::vector<std::thread> threads_;
  std::mutex mu_, region_;
  std::condition_variable cv_, done_;
  const std::function<void(int64_t)>* fn_ = nullptr;
  int64_t begin_ = 0, n_ = 0;
  int nt_ = 1, pending_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

inline void parallel_for(int64_t begin, int64_t end, const std::function<void(int64_t)>& fn,
                         int64_t min_per_thread = 1) {
  HostPool::get().run(begin, end, fn, min_per_thread);
}

// cos/sin of theta = pi * num / (2L-1), evaluated through the complement
// pi - theta so that the south pole (num = 2L-1) is exact.
inline void ring_trig(int L, int num, double* c, double* s, double* ch, double* sh) {
  const double D = 2.0 * L - 1.0;
  const double comp = (D - (double)num) / D;  // (pi - theta) / pi
  const double pi = 3.14159265358979323846;
  if (c) *c = -std::cos(pi * comp);
  if (s) *s = std::sin(pi * comp);
  if (ch) *ch = std::sin(0.5 * pi * comp);
  if (sh) *sh = std::cos(0.5 * pi * comp);
}

// Scaled associated Legendre values Pt[l, m](theta) = Y_l^m(theta, 0) for
// l = m..L-1 (m >= 0) at one colatitude, written to out[0 .. L-m-1].
// Seed Pt[m, m] by the product  Pt[i, i] = -sqrt((2i+1)/(2i)) sin(theta)
// Pt[i-1, i-1] from Pt[0, 0] = 1/sqrt(4 pi); then the normalised upward
// recurrence in l.  Values are carried as mantissa * 2^e so that seeds far
// below the double range still recur into range.
inline void legendre_order_host(int L, int m, double cs, double sn, double* out) {
  const double big = std::ldexp(1.0, 256), small = std::ldexp(1.0, -256);
  double p = 0.28209479177387814347;  // 1/sqrt(4 pi)
  int e = 0;
  for (int i = 1; i <= m; ++i) {
    p *= -std::sqrt((2.0 * i + 1.0) / (2.0 * i)) * sn;
    if (p == 0.0) break;
    if (std::fabs(p) < small) {
      int de;
      p = std::frexp(p, &de);
      e += de;
    }
  }
  double prev = 0.0, cur = p;
  out[0] = std::ldexp(cur, e);
  for (int l = m; l < L - 1; ++l) {
    const double den = (double)(l + 1) * (l + 1) - (double)m * m;
    const double a = std::sqrt((2.0 * l + 1.0) * (2.0 * l + 3.0) / den);
    const double b = (l == m) ? 0.0
        : std::sqrt((2.0 * l + 3.0) * ((double)l * l - (double)m * m) / ((2.0 * l - 1.0) * den));
    const double nxt = a * cs * cur - b * prev;
    prev = cur;
    cur = nxt;
    const double mag = std::max(std::fabs(prev), std::fabs(cur));
    if (mag > big) {
      prev *= small; cur *= small; e += 256;
    } else if (mag < small && mag > 0.0) {
      prev *= big; cur *= big; e -= 256;
    }
    out[l + 1 - m] = std::ldexp(cur, e);
  }
}

}  // namespace osht
