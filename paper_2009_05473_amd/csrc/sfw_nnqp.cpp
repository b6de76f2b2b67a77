// Non-negative quadratic program of the weights-only LASSO (algorithm 2, step 3 of BSFW; the
// weight step of SFW): minimise 1/2 w'Gw - c'w subject to w >= 0, with G the Gram matrix of
// the atoms' columns and c = Phi_k' y - lambda (section 1.1, the criterion restricted to the
// weights). Host code, float64; k is the support size (tens of atoms), so dense factorisations
// of k x k matrices are cheap next to the volume work that builds G.
#include <algorithm>
#include <cmath>
#include <vector>

#include "sfw.h"

namespace sfw {

namespace {

// Cholesky A = U'U of the s x s symmetric matrix given by its upper triangle (row-major); U
// overwrites that triangle. Right-looking, so every update is an AXPY over a contiguous row
// segment. False if A is not positive definite.
bool cholesky_upper(double* A, int s) {
  for (int j = 0; j < s; ++j) {
    double* rj = A + (size_t)j * s;
    const double d = rj[j];
    if (!(d > 0.0)) return false;
    const double u = std::sqrt(d);
    const double inv = 1.0 / u;
    rj[j] = u;
    for (int k = j + 1; k < s; ++k) rj[k] *= inv;
    for (int i = j + 1; i < s; ++i) {
      double* ri = A + (size_t)i * s;
      const double f = rj[i];
      for (int k = i; k < s; ++k) ri[k] -= f * rj[k];
    }
  }
  return true;
}

// Solves U'U x = b in place.
void chol_solve_upper(const double* U, int s, double* b) {
  for (int i = 0; i < s; ++i) {  // U' t = b (column i of U' is row i of U)
    const double t = b[i] / U[(size_t)i * s + i];
    b[i] = t;
    const double* ri = U + (size_t)i * s;
    for (int k = i + 1; k < s; ++k) b[k] -= ri[k] * t;
  }
  for (int i = s - 1; i >= 0; --i) {  // U x = t
    const double* ri = U + (size_t)i * s;
    double v = b[i];
    for (int k = i + 1; k < s; ++k) v -= ri[k] * b[k];
    b[i] = v / ri[i];
  }
}

// z_P = G_PP^{-1} c_P, z = 0 off P (ridge added if G_PP is singular, as duplicate atoms make
// it). A and L are scratch of at least |P|^2 entries.
void solve_passive(const std::vector<double>& G, const std::vector<double>& c, int k,
                   const std::vector<int>& P, std::vector<double>& z, std::vector<double>& A,
                   std::vector<double>& L, std::vector<double>& b) {
  const int s = (int)P.size();
  A.resize((size_t)s * s);
  L.resize((size_t)s * s);
  b.resize(s);
  double tr = 0.0;
  for (int i = 0; i < s; ++i) {
    const double* gi = G.data() + (size_t)P[i] * k;
    for (int j = i; j < s; ++j) A[(size_t)i * s + j] = gi[P[j]];
    b[i] = c[P[i]];
    tr += A[(size_t)i * s + i];
  }
  std::copy(A.begin(), A.end(), L.begin());
  if (!cholesky_upper(L.data(), s)) {
    const double ridge[2] = {1e-12 * tr / std::max(s, 1), 1e-6 * tr / std::max(s, 1)};
    for (double r : ridge) {
      std::copy(A.begin(), A.end(), L.begin());
      for (int i = 0; i < s; ++i) L[(size_t)i * s + i] += r;
      if (cholesky_upper(L.data(), s)) break;
    }
  }
  chol_solve_upper(L.data(), s, b.data());
  z.assign(k, 0.0);
  for (int i = 0; i < s; ++i) z[P[i]] = b[i];
}

}  // namespace

int nnqp(const std::vector<double>& G, const std::vector<double>& c, int k,
         std::vector<double>& w) {
  w.assign(k, 0.0);
  if (k == 0) return SFW_OK;
  std::vector<double> z, A, L, b;
  std::vector<int> P;
  std::vector<char> passive(k, 1);
  auto passive_set = [&]() {
    P.clear();
    for (int i = 0; i < k; ++i)
      if (passive[i]) P.push_back(i);
  };
  // Phase 1: supports usually keep most weights positive (zero-weight atoms are pruned), so
  // start from the full set and drop every coordinate whose solution is not positive until the
  // solution on the remaining set is. That point is feasible; if every weight stayed, the
  // gradient vanishes everywhere, the KKT conditions hold and (strictly convex objective) it is
  // the minimiser.
  for (int round = 0; round < k; ++round) {
    passive_set();
    if (P.empty()) break;
    solve_passive(G, c, k, P, z, A, L, b);
    bool positive = true;
    for (int i : P)
      if (!(z[i] > 0.0)) {
        passive[i] = 0;
        positive = false;
      }
    if (positive) {
      w = z;
      break;
    }
  }
  // Phase 2: Lawson-Hanson active set from the feasible point (w, passive): free the
  // coordinate with the most negative gradient, solve on the passive set and step back to
  // feasibility until the KKT conditions hold.
  double scale = 0.0;
  for (int i = 0; i < k; ++i) scale = std::max(scale, std::fabs(c[i]));
  const double tol = 1e-13 * std::max(scale, 1e-300);
  for (int outer = 0; outer < 4 * k + 20; ++outer) {
    // gradient of 1/2 w'Gw - c'w
    int jbest = -1;
    double gbest = -tol;
    for (int i = 0; i < k; ++i) {
      if (passive[i]) continue;
      double g = -c[i];
      for (int j = 0; j < k; ++j) g += G[(size_t)i * k + j] * w[j];
      if (g < gbest) {
        gbest = g;
        jbest = i;
      }
    }
    if (jbest < 0) return SFW_OK;
    passive[jbest] = 1;
    for (int inner = 0; inner < 4 * k + 20; ++inner) {
      passive_set();
      solve_passive(G, c, k, P, z, A, L, b);
      bool feasible = true;
      for (int i : P)
        if (!(z[i] > 0.0)) feasible = false;
      if (feasible) {
        w = z;
        break;
      }
      double alpha = 1.0;
      for (int i : P)
        if (!(z[i] > 0.0)) {
          const double den = w[i] - z[i];
          const double a = den > 0.0 ? w[i] / den : 0.0;
          alpha = std::min(alpha, a);
        }
      for (int i = 0; i < k; ++i) w[i] += alpha * (z[i] - w[i]);
      bool moved = false;
      for (int i : P)
        if (w[i] <= 1e-15 * std::max(1.0, std::fabs(z[i]))) {
          passive[i] = 0;
          w[i] = 0.0;
          moved = true;
        }
      if (!moved) {  // numerically stuck: drop the most negative member
        int worst = P[0];
        for (int i : P)
          if (z[i] < z[worst]) worst = i;
        passive[worst] = 0;
        w[worst] = 0.0;
      }
    }
  }
  return SFW_OK;
}

}  // namespace sfw
