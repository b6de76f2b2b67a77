// Host-only check of the library's non-negative quadratic program (the LASSO weight step,
// Algorithm 1 step 3 / Algorithm 2 step 3): min_{w >= 0} 1/2 w^T G w - c^T w for random
// symmetric positive definite G. Built with the sanitizers by tests/test_host_sanitized.py.
// Checks the KKT conditions of every solution: w >= 0, (G w - c)_i = 0 where w_i > 0 and
// >= 0 where w_i = 0 (relative 1e-9). Prints "ok <problems>" and returns 0 when all hold.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

namespace sfw {
int nnqp(const std::vector<double>& G, const std::vector<double>& c, int k, std::vector<double>& w);
}

int main() {
  std::mt19937_64 rng(12345);
  std::normal_distribution<double> nd(0.0, 1.0);
  int problems = 0;
  for (int k : {1, 2, 3, 5, 8, 13, 21, 34, 55, 89}) {
    for (int rep = 0; rep < 4; ++rep) {
      // G = A^T A + 1e-3 I with A of k + 3 rows: positive definite, condition moderate
      const int m = k + 3;
      std::vector<double> A((size_t)m * k), G((size_t)k * k, 0.0), c(k);
      for (double& a : A) a = nd(rng);
      for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
          double s = 0.0;
          for (int r = 0; r < m; ++r) s += A[(size_t)r * k + i] * A[(size_t)r * k + j];
          G[(size_t)i * k + j] = s + (i == j ? 1e-3 : 0.0);
        }
      for (double& v : c) v = nd(rng) * std::sqrt((double)m);
      std::vector<double> w;
      if (sfw::nnqp(G, c, k, w) != 0 || (int)w.size() != k) {
        std::printf("nnqp failed at k = %d\n", k);
        return 1;
      }
      double scale = 0.0;
      for (double v : c) scale = std::fmax(scale, std::fabs(v));
      for (int i = 0; i < k; ++i) {
        double g = -c[i];
        for (int j = 0; j < k; ++j) g += G[(size_t)i * k + j] * w[j];
        const double tol = 1e-9 * (scale + 1.0);
        if (w[i] < 0.0 || (w[i] > 0.0 && std::fabs(g) > tol) || (w[i] == 0.0 && g < -tol)) {
          std::printf("KKT violated at k = %d, i = %d: w = %.3e, grad = %.3e\n", k, i, w[i], g);
          return 1;
        }
      }
      ++problems;
    }
  }
  std::printf("ok %d\n", problems);
  return 0;
}
