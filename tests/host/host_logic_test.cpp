// Checks of the library's host-side logic against brute force, built with a
// plain C++ compiler under AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_logic.py.  Exit status 0 when every check holds.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <set>
#include <vector>

#include "host_logic.hpp"

using namespace amm;

static int failures = 0;
#define CHECK(cond, ...)                        \
  do {                                          \
    if (!(cond)) {                              \
      ++failures;                               \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);        \
      std::fprintf(stderr, "\n");               \
    }                                           \
  } while (0)

// Best (total, size) over every frequency set closed under k -> n-k with at most K members.
static std::pair<double, size_t> brute_closed(const std::vector<double>& E, int K) {
  const int n = (int)E.size();
  std::vector<std::vector<int>> classes;
  std::vector<bool> seen(n, false);
  for (int k = 0; k < n; ++k) {
    if (seen[k]) continue;
    const int kk = (n - k) % n;
    seen[k] = seen[kk] = true;
    classes.push_back(k == kk ? std::vector<int>{k} : std::vector<int>{k, kk});
  }
  double best = -1.0;
  size_t best_size = 0;
  const int c = (int)classes.size();
  for (int mask = 0; mask < (1 << c); ++mask) {
    double tot = 0.0;
    size_t size = 0;
    for (int i = 0; i < c; ++i)
      if (mask >> i & 1) {
        size += classes[i].size();
        for (int m : classes[i]) tot += E[m];
      }
    if ((int)size > K) continue;
    if (tot > best + 1e-12 || (std::fabs(tot - best) <= 1e-12 && size > best_size)) {
      best = tot;
      best_size = size;
    }
  }
  return {best, best_size};
}

static void test_select_closed(std::mt19937_64& g) {
  std::uniform_real_distribution<double> U(0.0, 1.0);
  for (int n = 1; n <= 12; ++n)
    for (int trial = 0; trial < 40; ++trial) {
      std::vector<double> E(n);
      for (double& e : E) e = (trial % 4 == 0) ? std::floor(U(g) * 3.0) : U(g);   // ties on some trials
      // a real operator's energies are mirror-symmetric
      for (int k = 1; k < n; ++k) E[n - k] = E[k];
      const std::vector<double> R = retained_all(E);
      for (int K = 0; K <= n; ++K) {
        const std::vector<int32_t> S = select_closed(E, K);
        CHECK((int)S.size() <= K, "n=%d K=%d size %zu", n, K, S.size());
        std::set<int> in(S.begin(), S.end());
        CHECK(in.size() == S.size() && std::is_sorted(S.begin(), S.end()), "n=%d K=%d not a sorted set", n, K);
        double tot = 0.0;
        for (int k : S) {
          CHECK(k >= 0 && k < n && in.count((n - k) % n), "n=%d K=%d not closed at %d", n, K, k);
          tot += E[k];
        }
        const auto b = brute_closed(E, K);
        CHECK(std::fabs(tot - b.first) <= 1e-12, "n=%d K=%d total %.17g best %.17g", n, K, tot, b.first);
        CHECK(std::fabs(tot - b.first) > 1e-12 || S.size() == b.second, "n=%d K=%d size %zu best %zu", n, K,
              S.size(), b.second);
        CHECK(std::fabs(R[K] - b.first) <= 1e-12, "n=%d K=%d retained %.17g best %.17g", n, K, R[K], b.first);
      }
    }
}

static void test_factorisations(std::mt19937_64& g) {
  std::normal_distribution<double> N(0.0, 1.0);
  for (int l : {1, 2, 5, 17, 48}) {
    std::vector<double> M(l * l), G(l * l, 0.0);
    for (double& v : M) v = N(g);
    for (int i = 0; i < l; ++i)
      for (int j = 0; j < l; ++j) {
        double s = 0.0;
        for (int k = 0; k < l; ++k) s += M[i * l + k] * M[j * l + k] * std::pow(k + 1.0, -1.0);
        G[i * l + j] = s + (i == j ? 1e-3 : 0.0);
      }
    double fro = 0.0;
    for (double v : G) fro += v * v;
    fro = std::sqrt(fro);
    // Cholesky and the triangular inverse
    std::vector<double> R = G;
    CHECK(cholesky_upper(R, l), "l=%d not positive definite", l);
    double err = 0.0;
    for (int i = 0; i < l; ++i)
      for (int j = 0; j < l; ++j) {
        if (j < i) CHECK(R[i * l + j] == 0.0, "l=%d lower part not zero", l);
        double s = 0.0;
        for (int k = 0; k < l; ++k) s += R[k * l + i] * R[k * l + j];
        err = std::max(err, std::fabs(s - G[i * l + j]));
      }
    CHECK(err <= 1e-12 * fro, "l=%d R^T R - G = %.3g", l, err);
    const std::vector<double> X = inv_upper(R, l);
    err = 0.0;
    for (int i = 0; i < l; ++i)
      for (int j = 0; j < l; ++j) {
        double s = 0.0;
        for (int k = 0; k < l; ++k) s += R[i * l + k] * X[k * l + j];
        err = std::max(err, std::fabs(s - (i == j ? 1.0 : 0.0)));
      }
    CHECK(err <= 1e-8, "l=%d R R^-1 - I = %.3g", l, err);
    // Jacobi eigen-decomposition: G W = W diag(lam), W orthogonal
    std::vector<double> lam, W;
    jacobi_eig(G, l, lam, W);
    double e1 = 0.0, e2 = 0.0;
    for (int i = 0; i < l; ++i)
      for (int j = 0; j < l; ++j) {
        double gw = 0.0, ww = 0.0;
        for (int k = 0; k < l; ++k) {
          gw += G[i * l + k] * W[k * l + j];
          ww += W[k * l + i] * W[k * l + j];
        }
        e1 = std::max(e1, std::fabs(gw - W[i * l + j] * lam[j]));
        e2 = std::max(e2, std::fabs(ww - (i == j ? 1.0 : 0.0)));
      }
    CHECK(e1 <= 1e-12 * fro && e2 <= 1e-12, "l=%d GW - W lam %.3g, W^T W - I %.3g", l, e1, e2);
  }
  // a singular matrix has no Cholesky factor
  std::vector<double> Z(9, 0.0);
  CHECK(!cholesky_upper(Z, 3), "zero matrix factored");
}

static void test_panels_overlap(std::mt19937_64& g) {
  static float buf[4096];
  for (int t = 0; t < 200000; ++t) {
    const int p = 1 + (int)(g() % 8), ld = p + (int)(g() % 6), ld2 = (g() % 4 == 0) ? ld + 1 : ld;
    const int ra = 1 + (int)(g() % 6), rb = 1 + (int)(g() % 6);
    const int oa = 2000, ob = oa + (int)(g() % 120) - 60;
    std::set<int> A;
    for (int i = 0; i < ra; ++i)
      for (int j = 0; j < p; ++j) A.insert(oa + i * ld + j);
    bool ov = false;
    for (int i = 0; i < rb; ++i)
      for (int j = 0; j < p; ++j) ov |= A.count(ob + i * ld2 + j) > 0;
    const bool got = panels_overlap(buf + oa, ra, ld, buf + ob, rb, ld2, p);
    if (ld2 == ld) CHECK(got == ov, "p=%d ld=%d ra=%d rb=%d d=%d: %d vs %d", p, ld, ra, rb, ob - oa, got, ov);
    else CHECK(got || !ov, "different pitches: overlap missed (p=%d d=%d)", p, ob - oa);   // conservative
  }
}

int main() {
  std::mt19937_64 g(20240419);
  test_select_closed(g);
  test_factorisations(g);
  test_panels_overlap(g);
  if (failures) {
    std::fprintf(stderr, "%d failure(s)\n", failures);
    return 1;
  }
  std::printf("host logic: all checks passed\n");
  return 0;
}
