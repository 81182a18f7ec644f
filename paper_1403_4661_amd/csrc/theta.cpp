// Colatitude placement of the L rings (Sec. III-D), computed on the host.
//
// Greedy: theta_{L-1} is the member of Theta = {pi (2t+1)/(2L-1)} farthest
// from the poles; for m = L-2 down to 0, theta_m is the unused member of
// Theta minimising cond_2(P_m), where P_m (Eq. Y_matrix) has the rows of
// rings m..L-1 and the columns of degrees m..L-1.  Ties (relative 1e-12)
// go to the smallest numerator.
//
// Evaluation: with B the n-1 fixed rows of P_m (n = L-m) and r a candidate
// row, cond_2([r; B])^2 = lam_max / lam_min of S + r r^T, S = B^T B.  S is
// reduced once per m to tridiagonal T = Q^T S Q by Householder reflections;
// each candidate is mapped to y = Q^T r, and the extreme eigenvalues of
// T + y y^T are the roots of the secular function
//     phi(lam) = 1 + y^T (T - lam I)^{-1} y
// in (0, mu_2) and (mu_n, mu_n + |y|^2), mu_i the eigenvalues of T (S has
// one zero eigenvalue because B has n-1 rows).  phi is evaluated by a
// tridiagonal solve with partial pivoting; phi' = |(T - lam)^{-1} y|^2 gives
// safeguarded Newton steps inside a shrinking bracket.  No eigenvectors are
// formed, so the cost per m is O(n^3) for S and T plus O(n) per evaluation.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "host_util.hpp"
#include "secular.hpp"

namespace osht {


// Greedy placement.  num_out[k] = n_k; kappa_out[m] = cond_2(P_m) (may be
// nullptr).  Returns 0.
int theta_greedy(int L, int32_t* num_out, double* kappa_out) {
  std::vector<int32_t> chosen(L, 0);
  std::vector<char> used(L, 0);
  std::vector<double> cs(L), sn(L);
  for (int t = 0; t < L; ++t) ring_trig(L, 2 * t + 1, &cs[t], &sn[t], nullptr, nullptr);
  chosen[L - 1] = 2 * ((L - 1) / 2) + 1;
  used[(chosen[L - 1] - 1) / 2] = 1;
  if (kappa_out) kappa_out[L - 1] = 1.0;
  std::vector<double> rows, S, av, bv;
  for (int m = L - 2; m >= 0; --m) {
    const int n = L - m;
    // rows[t * n + i] = Pt[m + i, m](theta of numerator 2t+1)
    rows.assign((size_t)L * n, 0.0);
    parallel_for(0, L, [&](int64_t t) { legendre_order_host(L, m, cs[t], sn[t], &rows[(size_t)t * n]); }, 8);
    // S = B^T B over the fixed rings m+1..L-1 (lower triangle by rank-1
    // accumulation over the rows of B, then mirrored)
    std::vector<const double*> fixed;
    for (int k = m + 1; k < L; ++k) fixed.push_back(&rows[(size_t)((chosen[k] - 1) / 2) * n]);
    S.assign((size_t)n * n, 0.0);
    parallel_for(0, n, [&](int64_t i) {
      double* si = &S[(size_t)i * n];
      for (const double* r : fixed) {
        const double ri = r[i];
        for (int j = 0; j <= i; ++j) si[j] += ri * r[j];
      }
    }, 4);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) S[(size_t)j * n + i] = S[(size_t)i * n + j];
    // Householder tridiagonalisation; reflector j (acting on rows/cols
    // j+1..n-1) is kept as v (v[0] = 1) with scale beta.
    av.assign(n, 0.0);
    bv.assign(std::max(n - 1, 1), 0.0);
    std::vector<std::vector<double>> vs;
    std::vector<double> betas;
    std::vector<double> p(n), w(n);
    for (int j = 0; j + 2 < n; ++j) {
      const int len = n - j - 1;
      std::vector<double> v(len);
      double sig = 0.0;
      for (int i = 0; i < len; ++i) {
        v[i] = S[(size_t)(j + 1 + i) * n + j];
        if (i > 0) sig += v[i] * v[i];
      }
      const double x0 = v[0];
      double beta = 0.0, alpha = x0;
      if (sig != 0.0) {
        const double nrm = std::sqrt(x0 * x0 + sig);
        alpha = (x0 <= 0.0) ? nrm : -nrm;  // H x = alpha e1
        const double v0 = x0 - alpha;
        beta = -v0 / alpha;  // 2 / (v^T v) with v scaled so v[0] = 1
        for (int i = 1; i < len; ++i) v[i] /= v0;
        v[0] = 1.0;
      }
      av[j] = S[(size_t)j * n + j];
      bv[j] = alpha;
      if (beta != 0.0) {
        // trailing block A22 <- H A22 H with H = I - beta v v^T
        parallel_for(0, len, [&](int64_t i) {
          const double* rowp = &S[(size_t)(j + 1 + i) * n + j + 1];
          double acc = 0.0;
          for (int k = 0; k < len; ++k) acc += rowp[k] * v[k];
          p[i] = beta * acc;
        }, 64);
        double pv = 0.0;
        for (int i = 0; i < len; ++i) pv += p[i] * v[i];
        const double half = 0.5 * beta * pv;
        for (int i = 0; i < len; ++i) w[i] = p[i] - half * v[i];
        parallel_for(0, len, [&](int64_t i) {
          double* rowp = &S[(size_t)(j + 1 + i) * n + j + 1];
          const double vi = v[i], wi = w[i];
          for (int k = 0; k < len; ++k) rowp[k] -= vi * w[k] + wi * v[k];
        }, 64);
      }
      vs.push_back(std::move(v));
      betas.push_back(beta);
    }
    if (n >= 2) {
      av[n - 2] = S[(size_t)(n - 2) * n + (n - 2)];
      av[n - 1] = S[(size_t)(n - 1) * n + (n - 1)];
      bv[n - 2] = S[(size_t)(n - 1) * n + (n - 2)];
    } else {
      av[0] = S[0];
    }
    // candidates, ascending numerators
    std::vector<int> cand;
    for (int t = 0; t < L; ++t) if (!used[t]) cand.push_back(t);
    const int nc = (int)cand.size();
    std::vector<double> kap(nc, std::numeric_limits<double>::infinity());
    if (n == 1) {
      for (int c = 0; c < nc; ++c) kap[c] = (rows[(size_t)cand[c] * n] != 0.0) ? 1.0 : INFINITY;
    } else {
      // mu1 is the (numerically tiny) zero eigenvalue of S; the smallest
      // eigenvalue of S + r r^T lies in (mu1, mu2), the largest in
      // (mun, mun + |r|^2).
      const double mu1 = secular::tri_eig(n, av.data(), bv.data(), 0);
      const double mu2 = secular::tri_eig(n, av.data(), bv.data(), 1);
      const double mun = secular::tri_eig(n, av.data(), bv.data(), n - 1);
      parallel_for(0, nc, [&](int64_t c) {
        std::vector<double> y(rows.begin() + (size_t)cand[c] * n, rows.begin() + (size_t)(cand[c] + 1) * n);
        std::vector<double> work(4 * n);
        double rr = 0.0;
        for (double v : y) rr += v * v;
        if (rr == 0.0) return;  // zero row: singular, kappa stays inf
        for (size_t j = 0; j < vs.size(); ++j) {  // y <- H_j y, j ascending
          const std::vector<double>& v = vs[j];
          if (betas[j] == 0.0) continue;
          double dot = 0.0;
          for (size_t i = 0; i < v.size(); ++i) dot += v[i] * y[j + 1 + i];
          dot *= betas[j];
          for (size_t i = 0; i < v.size(); ++i) y[j + 1 + i] -= dot * v[i];
        }
        kap[c] = secular::candidate_kappa(n, av.data(), bv.data(), secular::View<const double>{y.data(), 1}, rr, mu1,
                                          mu2, mun, secular::View<double>{work.data(), 1});
      }, 1);
    }
    double kmin = INFINITY;
    for (double k : kap) kmin = std::min(kmin, k);
    int pick = 0;
    for (int c = 0; c < nc; ++c) if (kap[c] <= kmin * (1.0 + 1e-12)) { pick = c; break; }
    chosen[m] = 2 * cand[pick] + 1;
    used[cand[pick]] = 1;
    if (kappa_out) kappa_out[m] = kap[pick];
  }
  for (int k = 0; k < L; ++k) num_out[k] = chosen[k];
  return 0;
}

void theta_alternating(int L, int32_t* num_out) {
  for (int k = 0; k < L; ++k) num_out[k] = (k % 2 == 0) ? (2 * L - 1 - k) : k;
}

}  // namespace osht
