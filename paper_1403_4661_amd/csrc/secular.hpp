// Tridiagonal and secular-equation helpers of the greedy colatitude placement
// (Sec. III-D), shared by the host greedy (theta.cpp) and its device twin
// (theta_gpu.hip) so that both evaluate cond_2 with the same operations in
// the same order.
//
// For B the n-1 fixed rows of P_m and r a candidate row,
// cond_2([r; B])^2 = lam_max / lam_min of S + r r^T with S = B^T B.  With
// S = Q T Q^T (T symmetric tridiagonal) and y = Q^T r, the extreme
// eigenvalues of T + y y^T are the roots of
//     phi(lam) = 1 + y^T (T - lam I)^{-1} y
// in (mu_1, mu_2) and (mu_n, mu_n + |y|^2), mu_i the eigenvalues of T.
#pragma once

#include <cfloat>
#include <cmath>
#include <cstdint>

#if defined(__HIP__)
#define OSHT_HD __host__ __device__
#else
#define OSHT_HD
#endif

namespace osht {
namespace secular {

// Strided view: element i at p[i * s] (s = 1 on the host; on the device the
// per-candidate arrays are interleaved so that a wave's accesses coalesce).
template <class T>
struct View {
  T* p;
  int64_t s;
  OSHT_HD T& operator[](int64_t i) const { return p[i * s]; }
};

// Solve (T - lam I) x = y for symmetric tridiagonal T (diagonal a[0..n-1],
// off-diagonal b[0..n-2]) by Gaussian elimination with partial pivoting.
// Returns y^T x and writes |x|^2 to *xx.  work: 4n entries.
OSHT_HD inline double tri_solve_dot(int n, const double* a, const double* b, double lam, View<const double> y,
                                    View<double> work, double* xx) {
#pragma clang fp contract(off)
  // work[0, n): pivot-row diagonal; [n, 2n): first super-diagonal;
  // [2n, 3n): second super-diagonal (from row swaps); [3n, 4n): transformed
  // right-hand side.  The back substitution carries x[i+1], x[i+2] in
  // registers, so its loads do not wait on its own stores.
  const int64_t U0 = 0, U1 = n, U2 = 2 * (int64_t)n, RH = 3 * (int64_t)n;
  const double tiny = DBL_MIN * 16;
  // current pivot-candidate row: (p0, p1, p2) at columns i, i+1, i+2
  double p0 = a[0] - lam, p1 = (n > 1) ? b[0] : 0.0, p2 = 0.0, prh = y[0];
#pragma unroll 4
  for (int i = 0; i < n - 1; ++i) {
    const double r0 = b[i];
    const double r1 = a[i + 1] - lam;
    const double r2 = (i + 1 < n - 1) ? b[i + 1] : 0.0;
    const double rrh = y[i + 1];
    if (fabs(p0) >= fabs(r0)) {
      const double piv = (p0 == 0.0) ? tiny : p0;
      const double f = r0 / piv;
      work[U0 + i] = piv; work[U1 + i] = p1; work[U2 + i] = p2; work[RH + i] = prh;
      p0 = r1 - f * p1; p1 = r2 - f * p2; p2 = 0.0; prh = rrh - f * prh;
    } else {
      const double f = p0 / r0;
      work[U0 + i] = r0; work[U1 + i] = r1; work[U2 + i] = r2; work[RH + i] = rrh;
      p0 = p1 - f * r1; p1 = p2 - f * r2; p2 = 0.0; prh = prh - f * rrh;
    }
  }
  work[U0 + n - 1] = (p0 == 0.0) ? tiny : p0;
  work[RH + n - 1] = prh;
  double dot = 0.0, nrm = 0.0, x1 = 0.0, x2 = 0.0;  // x[i+1], x[i+2]
#pragma unroll 4
  for (int i = n - 1; i >= 0; --i) {
    double v = work[RH + i];
    if (i + 1 < n) v -= work[U1 + i] * x1;
    if (i + 2 < n) v -= work[U2 + i] * x2;
    const double xi = v / work[U0 + i];
    dot += y[i] * xi;
    nrm += xi * xi;
    x2 = x1;
    x1 = xi;
  }
  *xx = nrm;
  return dot;
}

// Number of eigenvalues of T below x (Sturm count from the LDL^T pivots).
OSHT_HD inline int sturm_count(int n, const double* a, const double* b, double x) {
#pragma clang fp contract(off)
  int cnt = 0;
  double q = a[0] - x;
  const double tiny = DBL_MIN * 16;
  if (q < 0) ++cnt;
  for (int i = 1; i < n; ++i) {
    if (q == 0.0) q = tiny;
    q = (a[i] - x) - b[i - 1] * b[i - 1] / q;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// k-th smallest eigenvalue of T (k = 0..n-1) by bisection on the Sturm count.
OSHT_HD inline double tri_eig(int n, const double* a, const double* b, int k) {
#pragma clang fp contract(off)
  double lo = a[0], hi = a[0];
  for (int i = 0; i < n; ++i) {
    double r = 0.0;
    if (i > 0) r += fabs(b[i - 1]);
    if (i < n - 1) r += fabs(b[i]);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
  }
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(n, a, b, mid) > k) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Root of phi(base + t) for t in (lo, hi), phi increasing there; geometric
// bisection in t when `geometric` is set (lo > 0), Newton steps when they
// stay in the bracket.  Returns base + t at the root.
OSHT_HD inline double secular_root(int n, const double* a, const double* b, View<const double> y, double base,
                                   double lo, double hi, bool geometric, View<double> work) {
#pragma clang fp contract(off)
  double t = geometric ? sqrt(lo * hi) : 0.5 * (lo + hi);
  for (int it = 0; it < 400; ++it) {
    double xx;
    const double phi = 1.0 + tri_solve_dot(n, a, b, base + t, y, work, &xx);
    if (phi == 0.0) return base + t;
    if (phi < 0.0) lo = t; else hi = t;
    if (hi - lo <= 4e-16 * hi) return base + 0.5 * (lo + hi);
    double nxt = t - phi / xx;  // phi' = |x|^2
    if (!(nxt > lo && nxt < hi)) {
      nxt = geometric ? sqrt(lo * hi) : 0.5 * (lo + hi);
    } else if (fabs(nxt - t) <= 4e-16 * fabs(t)) {
      return base + nxt;  // Newton has converged to rounding level
    }
    t = nxt;
  }
  return base + t;
}

// cond_2([r; B]) for one candidate from y = Q^T r, the tridiagonal T of
// S = B^T B and its eigenvalues mu1 <= mu2 (smallest two) and mun
// (largest); rr = |r|^2.  Infinity for a zero row or when the computed
// spectrum carries no information (kappa above ~1e7 reads as singular).
OSHT_HD inline double candidate_kappa(int n, const double* a, const double* b, View<const double> y, double rr,
                                      double mu1, double mu2, double mun, View<double> work) {
#pragma clang fp contract(off)
  if (rr == 0.0) return INFINITY;
  const double gap = mu2 - mu1;
  // below ~1e-15 |S| the computed spectrum carries no information
  const double t_lo = fmax(gap * ldexp(1.0, -200), 1e-15 * mun);
  double xx;
  if (1.0 + tri_solve_dot(n, a, b, mu1 + t_lo, y, work, &xx) >= 0.0) return INFINITY;
  const double lmin = secular_root(n, a, b, y, mu1, t_lo, gap, true, work) - mu1;
  const double lmax = secular_root(n, a, b, y, mun, 0.0, rr * (1 + 1e-12) + 1e-300, false, work);
  return sqrt(lmax / lmin);
}

}  // namespace secular
}  // namespace osht
