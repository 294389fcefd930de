// Host-side logic with no device code (see host_logic.hpp).
#include "host_logic.hpp"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

namespace amm {

std::vector<int32_t> select_closed(const std::vector<double>& E, int K) {
  // Among frequency sets closed under k -> n-k with at most K members, keep
  // the one with the largest total energy.  Singleton classes are {0} and
  // {n/2}; every other class is a pair, so for each subset of singletons the
  // best completion is the top pairs by E[k] + E[n-k] (ties: smaller k).
  const int n = (int)E.size();
  std::vector<int> singles{0};
  if (n % 2 == 0 && n > 1) singles.push_back(n / 2);
  std::vector<int> pairs;
  for (int k = 1; k < (n + 1) / 2; ++k) pairs.push_back(k);
  std::stable_sort(pairs.begin(), pairs.end(), [&](int a, int b) {
    const double ea = E[a] + E[n - a], eb = E[b] + E[n - b];
    if (ea != eb) return ea > eb;
    return a < b;
  });
  std::vector<std::vector<int>> subsets{{}};
  for (int sgl : singles) subsets.push_back({sgl});
  if (singles.size() == 2) subsets.push_back(singles);
  bool have = false;
  double best_total = 0.0;
  size_t best_size = 0;
  std::vector<int32_t> best;
  for (const auto& U : subsets) {
    if ((int)U.size() > K) continue;
    std::vector<int32_t> members(U.begin(), U.end());
    const int np = (K - (int)U.size()) / 2;
    for (int i = 0; i < np && i < (int)pairs.size(); ++i) {
      members.push_back(pairs[i]);
      members.push_back(n - pairs[i]);
    }
    double total = 0.0;
    for (int m : members) total += E[m];
    if (!have || total > best_total || (total == best_total && members.size() > best_size)) {
      have = true;
      best_total = total;
      best_size = members.size();
      best = members;
    }
  }
  std::sort(best.begin(), best.end());
  return best;
}

std::vector<double> retained_all(const std::vector<double>& E) {
  // R[K] = energy kept by select_closed(E, K) for K = 0..n, from prefix sums of
  // the sorted pair energies (the same candidate sets as select_closed)
  const int n = (int)E.size();
  std::vector<int> singles{0};
  if (n % 2 == 0 && n > 1) singles.push_back(n / 2);
  std::vector<double> pe;
  for (int k = 1; k < (n + 1) / 2; ++k) pe.push_back(E[k] + E[n - k]);
  std::sort(pe.begin(), pe.end(), [](double a, double b) { return a > b; });
  std::vector<double> pre(pe.size() + 1, 0.0);
  for (size_t i = 0; i < pe.size(); ++i) pre[i + 1] = pre[i] + pe[i];
  std::vector<std::pair<int, double>> subsets{{0, 0.0}};
  for (int sgl : singles) subsets.push_back({1, E[sgl]});
  if (singles.size() == 2) subsets.push_back({2, E[singles[0]] + E[singles[1]]});
  std::vector<double> R(n + 1, 0.0);
  for (int K = 0; K <= n; ++K) {
    double best = 0.0;
    for (const auto& u : subsets) {
      if (u.first > K) continue;
      const size_t np = std::min<size_t>((size_t)(K - u.first) / 2, pe.size());
      best = std::max(best, u.second + pre[np]);
    }
    R[K] = best;
  }
  return R;
}

// Cholesky G = R^T R (upper R); returns false if not positive definite.
bool cholesky_upper(std::vector<double>& G, int l) {
  for (int j = 0; j < l; ++j) {
    double d = G[j * l + j];
    for (int k = 0; k < j; ++k) d -= G[k * l + j] * G[k * l + j];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    G[j * l + j] = d;
    for (int i = j + 1; i < l; ++i) {
      double v = G[j * l + i];
      for (int k = 0; k < j; ++k) v -= G[k * l + j] * G[k * l + i];
      G[j * l + i] = v / d;
    }
    for (int i = 0; i < j; ++i) G[j * l + i] = 0.0;
  }
  return true;
}

// inverse of an upper-triangular R (row-major)
std::vector<double> inv_upper(const std::vector<double>& R, int l) {
  std::vector<double> X(l * l, 0.0);
  for (int j = 0; j < l; ++j) {
    X[j * l + j] = 1.0 / R[j * l + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += R[i * l + k] * X[k * l + j];
      X[i * l + j] = -s / R[i * l + i];
    }
  }
  return X;
}

// cyclic Jacobi: G = W diag(lam) W^T
void jacobi_eig(std::vector<double> G, int l, std::vector<double>& lam, std::vector<double>& W) {
  W.assign(l * l, 0.0);
  for (int i = 0; i < l; ++i) W[i * l + i] = 1.0;
  double fro = 0.0;
  for (double v : G) fro += v * v;
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < l; ++i)
      for (int j = i + 1; j < l; ++j) off += G[i * l + j] * G[i * l + j];
    if (std::sqrt(off) <= 1e-16 * fro) break;
    for (int p = 0; p < l; ++p)
      for (int q = p + 1; q < l; ++q) {
        const double apq = G[p * l + q];
        if (apq == 0.0) continue;
        const double app = G[p * l + p], aqq = G[q * l + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < l; ++k) {
          const double gkp = G[k * l + p], gkq = G[k * l + q];
          G[k * l + p] = c * gkp - s * gkq;
          G[k * l + q] = s * gkp + c * gkq;
        }
        for (int k = 0; k < l; ++k) {
          const double gpk = G[p * l + k], gqk = G[q * l + k];
          G[p * l + k] = c * gpk - s * gqk;
          G[q * l + k] = s * gpk + c * gqk;
        }
        for (int k = 0; k < l; ++k) {
          const double wkp = W[k * l + p], wkq = W[k * l + q];
          W[k * l + p] = c * wkp - s * wkq;
          W[k * l + q] = s * wkp + c * wkq;
        }
      }
  }
  lam.resize(l);
  for (int i = 0; i < l; ++i) lam[i] = G[i * l + i];
}

// Whether two row panels of p floats (rows at a + i lda, i < ra, and at
// b + k ldb, k < rb) share an element.  With one pitch and a whole-float
// offset the test is exact (panels side by side in one matrix are disjoint);
// otherwise the address ranges must be disjoint.
bool panels_overlap(const float* a, int64_t ra, int64_t lda, const float* b, int64_t rb, int64_t ldb, int64_t p) {
  const intptr_t diff = (intptr_t)b - (intptr_t)a;
  if (lda == ldb && diff % (intptr_t)sizeof(float) == 0) {
    const int64_t ld = lda, d = diff / (intptr_t)sizeof(float);
    int64_t q = d / ld, r = d % ld;   // b = a + q ld + r, 0 <= r < ld
    if (r < 0) {
      r += ld;
      q -= 1;
    }
    auto rows_meet = [&](int64_t lo) { return lo < ra && lo + rb > 0; };   // [lo, lo + rb) against [0, ra)
    return (r < p && rows_meet(q)) || (ld - r < p && rows_meet(q + 1));
  }
  const uintptr_t a0 = (uintptr_t)a, a1 = a0 + (uintptr_t)((ra - 1) * lda + p) * sizeof(float);
  const uintptr_t b0 = (uintptr_t)b, b1 = b0 + (uintptr_t)((rb - 1) * ldb + p) * sizeof(float);
  return a0 < b1 && b0 < a1;
}

}  // namespace amm
