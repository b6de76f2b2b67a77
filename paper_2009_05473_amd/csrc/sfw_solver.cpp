// sfw_solve: SFW (algorithm 1) and BSFW (algorithm 2) driven from the host in float64, with
// every volume operation (render, blur, residual, adjoint, gradient sums, grid certificate,
// LASSO columns and Gram entries) on the GPU through the operator layer.
//
// Local ascent of eta (step 1) and the sliding descent of C (SFW step 4, BSFW step 2b) use a
// box-bounded limited-memory BFGS; the weights-only LASSO (step 3) is a non-negative
// quadratic program solved by a primal active-set method.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <limits>
#include <string>
#include <utility>
#include <vector>

#include "sfw_internal.h"
#include "sfw_ops.h"

// Slope-only steps without a halving of the projected gradient before a sliding descent stops
#ifndef SFW_SLOPE_STALL
#define SFW_SLOPE_STALL 30
#endif

namespace sfw {

namespace {

using Clock = std::chrono::steady_clock;
double secs(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double>(b - a).count();
}

}  // namespace

namespace {

// ------------------------------------------------------------------ box-bounded L-BFGS

struct MinResult {
  int iterations = 0;
  int evaluations = 0;
  bool converged = false;
  double f = 0.0;
  int status = SFW_OK;
  const char* stop = "iterations";  // why the descent stopped (verbose output)
};

using FG = std::function<int(const std::vector<double>&, double&, std::vector<double>&)>;

// Relative resolution of a value the library computes (criterion, certificate): float32
// voxels summed in float64.
constexpr double kFloat32Resolution = 1e-7;

// noise_stop: end the line search once the predicted decrease is below the float32
// resolution of f (used for the local ascent, whose result only seeds a new mass; the
// sliding descents keep backtracking, which lets nearby masses finish merging).
// slope_tol > 0 (the sliding descents): f comes from float32 volumes, so near a minimum its
// decrease along a step sinks below f's own rounding (relative ~1e-7 to 1e-6) long before the
// gradient, a float64 sum over many voxels, stops resolving the minimum. A step that fails the
// sufficient-decrease test is then still taken when f stays within slope_tol |f| of its old
// value and the slope along the step has not changed sign beyond the approximate Wolfe bound
// of Hager and Zhang (2005): phi'(a) <= (2 delta - 1) phi'(0) with delta = 0.1. Once such
// slope-only steps stop shrinking the projected gradient (no halving in kSlopeStall steps), the
// descent has reached the working precision of the gradient and stops.
MinResult minimize_box(const FG& fg, std::vector<double>& x, const std::vector<double>& lo,
                       const std::vector<double>& hi, int m, double gtol, double ftol,
                       int maxiter, bool noise_stop = false, double slope_tol = 0.0) {
  constexpr int kSlopeStall = SFW_SLOPE_STALL;
  double pg_ref = std::numeric_limits<double>::infinity();
  int stall = 0;
  MinResult res;
  const int n = (int)x.size();
  for (int i = 0; i < n; ++i) x[i] = std::min(std::max(x[i], lo[i]), hi[i]);
  std::vector<double> g(n), gn(n), xn(n), d(n);
  double f = 0.0, fnew = 0.0;
  int rc = fg(x, f, g);
  res.evaluations = 1;
  if (rc) {
    res.status = rc;
    return res;
  }
  std::deque<std::vector<double>> S, Y;
  std::deque<double> RHO;
  auto at_lo = [&](int i, const std::vector<double>& gg) { return x[i] <= lo[i] && gg[i] > 0; };
  auto at_hi = [&](int i, const std::vector<double>& gg) { return x[i] >= hi[i] && gg[i] < 0; };
  for (int it = 0; it < maxiter; ++it) {
    double pgmax = 0.0;
    std::vector<char> freev(n);
    for (int i = 0; i < n; ++i) {
      freev[i] = !(at_lo(i, g) || at_hi(i, g));
      if (freev[i]) pgmax = std::max(pgmax, std::fabs(g[i]));
    }
    res.iterations = it;
    if (pgmax <= gtol) {
      res.converged = true;
      res.stop = "gtol";
      break;
    }
    if (pgmax < 0.5 * pg_ref) {
      pg_ref = pgmax;
      stall = 0;
    }
    // two-loop recursion on the free coordinates
    for (int i = 0; i < n; ++i) d[i] = freev[i] ? -g[i] : 0.0;
    const int ms = (int)S.size();
    std::vector<double> alpha(ms);
    for (int j = ms - 1; j >= 0; --j) {
      double a = 0.0;
      for (int i = 0; i < n; ++i)
        if (freev[i]) a += S[j][i] * d[i];
      a *= RHO[j];
      alpha[j] = a;
      for (int i = 0; i < n; ++i)
        if (freev[i]) d[i] -= a * Y[j][i];
    }
    if (ms > 0) {
      double sy = 0.0, yy = 0.0;
      for (int i = 0; i < n; ++i) {
        sy += S[ms - 1][i] * Y[ms - 1][i];
        yy += Y[ms - 1][i] * Y[ms - 1][i];
      }
      const double gam = yy > 0 ? sy / yy : 1.0;
      for (int i = 0; i < n; ++i) d[i] *= gam;
    }
    for (int j = 0; j < ms; ++j) {
      double b = 0.0;
      for (int i = 0; i < n; ++i)
        if (freev[i]) b += Y[j][i] * d[i];
      b *= RHO[j];
      for (int i = 0; i < n; ++i)
        if (freev[i]) d[i] += S[j][i] * (alpha[j] - b);
    }
    double gd = 0.0, gg = 0.0;
    for (int i = 0; i < n; ++i) {
      if (!freev[i]) d[i] = 0.0;
      gd += g[i] * d[i];
      if (freev[i]) gg += g[i] * g[i];
    }
    if (!(gd < 0.0)) {  // not a descent direction: restart from steepest descent
      S.clear();
      Y.clear();
      RHO.clear();
      for (int i = 0; i < n; ++i) d[i] = freev[i] ? -g[i] : 0.0;
      gd = -gg;
    }
    double step = 1.0;
    if (S.empty()) {
      double dmax = 0.0;
      for (int i = 0; i < n; ++i) dmax = std::max(dmax, std::fabs(d[i]));
      step = dmax > 0 ? std::min(1.0, 1.0 / dmax) : 1.0;
    }
    bool accepted = false, by_slope = false;
    for (int ls = 0; ls < 40; ++ls) {
      double dec = 0.0;
      for (int i = 0; i < n; ++i) {
        xn[i] = std::min(std::max(x[i] + step * d[i], lo[i]), hi[i]);
        dec += g[i] * (xn[i] - x[i]);
      }
      // f is evaluated from float32 volumes: once the predicted decrease is below its
      // resolution, no sufficient-decrease test can be trusted; stop backtracking
      if (noise_stop && -dec <= kFloat32Resolution * std::max(std::fabs(f), 1.0)) break;
      rc = fg(xn, fnew, gn);
      res.evaluations++;
      if (rc) {
        res.status = rc;
        return res;
      }
      if (std::isfinite(fnew) && fnew <= f + 1e-4 * dec) {
        accepted = true;
        break;
      }
      if (slope_tol > 0 && std::isfinite(fnew) &&
          fnew <= f + slope_tol * std::max(std::fabs(f), 1.0)) {
        double dnew = 0.0;  // slope at the new point along the step taken
        for (int i = 0; i < n; ++i) dnew += gn[i] * (xn[i] - x[i]);
        if (dnew <= -0.8 * dec) {
          accepted = by_slope = true;
          break;
        }
      }
      step *= (ls < 2 ? 0.5 : 0.25);
    }
    if (!accepted) {
      if (S.empty()) {  // even a steepest-descent step fails: stationary to working precision
        res.converged = true;
        res.stop = "no descent step";
        break;
      }
      S.clear();
      Y.clear();
      RHO.clear();
      continue;
    }
    std::vector<double> s(n), yv(n);
    double sy = 0.0, ss = 0.0, yy = 0.0;
    for (int i = 0; i < n; ++i) {
      s[i] = xn[i] - x[i];
      yv[i] = gn[i] - g[i];
      sy += s[i] * yv[i];
      ss += s[i] * s[i];
      yy += yv[i] * yv[i];
    }
    const bool small_dec = (f - fnew) <= ftol * std::max(std::max(std::fabs(f), std::fabs(fnew)), 1.0);
    x = xn;
    g = gn;
    f = fnew;
    if (sy > 1e-12 * std::sqrt(ss * yy) && sy > 0) {
      S.push_back(s);
      Y.push_back(yv);
      RHO.push_back(1.0 / sy);
      if ((int)S.size() > m) {
        S.pop_front();
        Y.pop_front();
        RHO.pop_front();
      }
    }
    if (by_slope && ++stall >= kSlopeStall) {  // the gradient's working precision
      res.iterations = it + 1;
      res.converged = true;
      res.stop = "slope stall";
      break;
    }
    if (small_dec && !by_slope) {
      res.iterations = it + 1;
      res.converged = true;
      res.stop = "small decrease";
      break;
    }
    res.iterations = it + 1;
  }
  res.f = f;
  return res;
}

// ------------------------------------------------------------------ solver state

struct Solver {
  sfw_workspace* ws;
  sfw_dims vol;
  sfw_dims psf;
  const float* y;
  const float* H;
  double lam;
  sfw_options o;
  PsfPlan plan;
  size_t V;
  sfw_stats st{};
  // atoms (w, mx, my, mz, sigma, d) in float64
  std::vector<double> atoms;
  int k() const { return (int)(atoms.size() / 6); }

  // The atoms' kernel constants (AtomK, from the float32 parameters the kernels see) into
  // ws->ak: computed here and copied, with no preparation kernel.
  int upload_atoms(const std::vector<double>& a, bool unit_weight) {
    const int n = (int)(a.size() / 6);
    if (n == 0) return SFW_OK;
    AtomK* h = reinterpret_cast<AtomK*>(ws->hpin + ws->hp_stage);
    for (int i = 0; i < n; ++i) {
      const double* p = &a[6 * i];
      h[i] = make_atomk(unit_weight ? 1.0 : (double)(float)p[0], (double)(float)p[1],
                        (double)(float)p[2], (double)(float)p[3], (double)(float)p[4],
                        (double)(float)p[5]);
    }
    SFW_HIP(hipMemcpyAsync(ws->ak, h, sizeof(AtomK) * n, hipMemcpyHostToDevice, ws->stream));
    // No wait here: the staging buffer is only rewritten by the next upload (or an eta
    // evaluation), and every caller synchronises the stream (its readback) before that, so the
    // copy has finished by then.
    return SFW_OK;
  }

  // C and dC/d(atoms) at a (float64 host), r and q left in the workspace.
  int cgrad(const std::vector<double>& a, double& C, std::vector<double>* grad) {
    const int n = (int)(a.size() / 6);
    int rc = upload_atoms(a, false);
    if (rc) return rc;
    // the sums land in pinned host memory straight from the finalize kernel
    double* hs = ws->hpin + ws->hp_sums;
    // no device atoms: the host adds lambda * sum w to the data term hs[6 n + 1]
    rc = op_cgrad(ws, plan, vol, y, (float)lam, nullptr, n, nullptr, nullptr, nullptr, hs);
    if (rc) return rc;
    rc = sig_wait(ws, ws->sums_sig);
    if (rc) return rc;
    st.n_eval_cgrad++;
    double wsum = 0.0;
    for (int i = 0; i < n; ++i) wsum += a[6 * i];
    C = hs[6 * n + 1] + lam * wsum;
    if (grad) {
      const double ln2 = 0.69314718055994531;
      grad->assign(6 * (size_t)n, 0.0);
      for (int i = 0; i < n; ++i) {
        const double* S = hs + 6 * i;
        const double w = a[6 * i], sg = a[6 * i + 4], d = a[6 * i + 5];
        double* g = grad->data() + 6 * i;
        g[0] = lam - S[0];
        g[1] = -w * d * ln2 * S[3];
        g[2] = -w * d * ln2 * S[4];
        g[3] = -w * d * ln2 * S[5];
        g[4] = -w * (d / sg) * ln2 * S[1];
        g[5] = w * (0.5 * ln2 * ln2 * S[2] - std::log(sg) * ln2 * S[1]);
      }
    }
    return SFW_OK;
  }

  void theta_bounds(std::vector<double>& lo, std::vector<double>& hi) const {
    lo = {0.0, 0.0, 0.0, (double)o.sigma_lo, (double)o.d_lo};
    hi = {vol.nx - 1.0, vol.ny - 1.0, vol.nz - 1.0, (double)o.sigma_hi, (double)o.d_hi};
  }

  int ascent(std::vector<double>& th, double& eta_star) {
    std::vector<double> lo, hi;
    theta_bounds(lo, hi);
    FG fg = [&](const std::vector<double>& x, double& f, std::vector<double>& g) -> int {
      double e;
      g.assign(5, 0.0);
      int rc = op_eta_points(ws, vol, ws->q, lam, x.data(), 1, &e, g.data());
      st.n_eval_eta++;
      f = -e;
      for (double& v : g) v = -v;
      return rc;
    };
    MinResult r = minimize_box(fg, th, lo, hi, o.lbfgs_memory, o.ascent_gtol, o.ftol,
                               o.ascent_max_iter, true);
    st.n_ascent_iterations += r.iterations;
    if (r.status) return r.status;
    eta_star = -r.f;  // the minimiser's last value is eta at the returned point
    return SFW_OK;
  }

  int slide() {
    const int n = k();
    if (n == 0) return SFW_OK;
    std::vector<double> lo(6 * (size_t)n), hi(6 * (size_t)n), tl, th;
    theta_bounds(tl, th);
    for (int i = 0; i < n; ++i) {
      lo[6 * i] = 0.0;
      hi[6 * i] = std::numeric_limits<double>::infinity();
      for (int c = 0; c < 5; ++c) {
        lo[6 * i + 1 + c] = tl[c];
        hi[6 * i + 1 + c] = th[c];
      }
    }
    FG fg = [&](const std::vector<double>& x, double& f, std::vector<double>& g) -> int {
      return cgrad(x, f, &g);
    };
    MinResult r = minimize_box(fg, atoms, lo, hi, o.lbfgs_memory, o.slide_gtol, o.ftol,
                               o.slide_max_iter, false, o.slide_slope_tol);
    st.n_slide_iterations += r.iterations;
    if (o.verbose)
      std::fprintf(stderr, "[sfw] slide n=%d it=%d evals=%d converged=%d (%s) C=%.12g\n", n,
                   r.iterations, r.evaluations, (int)r.converged, r.stop, r.f);
    return r.status;
  }

  // Weights of the current support by the LASSO (the workspace reuses the columns of the
  // unchanged prefix of the support).
  int lasso() {
    const int n = k();
    if (n == 0) return SFW_OK;
    std::vector<float> th(5 * (size_t)n);
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < 5; ++c) th[5 * i + c] = (float)atoms[6 * i + 1 + c];
    std::vector<double> w;
    int rc = op_lasso(ws, plan, vol, y, H, lam, th.data(), n, w);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) atoms[6 * i] = w[i];
    return SFW_OK;
  }

  // Remove zero-weighted masses and merge coincident ones.
  void prune() {
    const int n = k();
    if (n == 0) return;
    double wmax = 0.0;
    for (int i = 0; i < n; ++i) wmax = std::max(wmax, atoms[6 * i]);
    std::vector<double> kept;
    int kept_n = 0;
    for (int i = 0; i < n; ++i) {
      const double* a = &atoms[6 * i];
      if (!(wmax > 0.0) || !(a[0] > o.prune_rel * wmax)) {
        continue;
      }
      bool merged = false;
      for (int j = 0; j < kept_n; ++j) {
        double* bj = &kept[6 * j];
        double dmax = 0.0;
        for (int c = 1; c < 6; ++c) dmax = std::max(dmax, std::fabs(a[c] - bj[c]));
        if (dmax <= o.merge_tol) {
          const double ws_ = a[0] + bj[0];
          if (ws_ > 0)
            for (int c = 1; c < 6; ++c) bj[c] = (bj[0] * bj[c] + a[0] * a[c]) / ws_;
          bj[0] = ws_;
          merged = true;
          break;
        }
      }
      if (!merged) {
        kept.insert(kept.end(), a, a + 6);
        kept_n++;
      }
    }
    atoms.swap(kept);
  }
};

}  // namespace

}  // namespace sfw

using namespace sfw;

extern "C" int sfw_solve(sfw_workspace* ws, const float* y, sfw_dims vol, const float* H,
                         sfw_dims psf, float lambda, const sfw_options* opts,
                         sfw_atom* atoms_out, int cap, int* n_out, sfw_stats* stats) {
  try {
    int rc = check_ws_fit(ws, vol, &psf, 0);
    if (rc) return rc;
    if (!y || !H) return fail(SFW_EINVAL, "y or H is NULL");
    if (!n_out) return fail(SFW_EINVAL, "n_out is NULL");
    if (cap < 0 || (cap > 0 && !atoms_out)) return fail(SFW_EINVAL, "atoms_out/cap invalid");
    rc = check_lambda(lambda);
    if (rc) return rc;
    Solver S;
    S.ws = ws;
    S.vol = vol;
    S.psf = psf;
    S.y = y;
    S.H = H;
    S.lam = lambda;
    if (opts)
      S.o = *opts;
    else
      sfw_default_options(&S.o);
    const sfw_options& o = S.o;
    if (o.mode != SFW_MODE_BSFW && o.mode != SFW_MODE_SFW)
      return fail(SFW_EINVAL, "opts.mode must be SFW_MODE_BSFW or SFW_MODE_SFW");
    if (o.n_sigma < 1 || o.n_sigma > SFW_MAX_GRID || o.n_d < 1 || o.n_d > SFW_MAX_GRID)
      return fail(SFW_EINVAL, "opts grid sizes must be in [1, SFW_MAX_GRID]");
    if (o.n_sigma * o.n_d > SFW_CERT_MAX_KERNELS)
      return fail(SFW_EINVAL, "opts.n_sigma * opts.n_d must be at most SFW_CERT_MAX_KERNELS");
    if (!(o.sigma_lo > 0) || !(o.sigma_hi >= o.sigma_lo) || !(o.d_lo > 0) || !(o.d_hi >= o.d_lo))
      return fail(SFW_EINVAL, "opts bounds of sigma / d invalid");
    for (int i = 0; i < o.n_sigma; ++i)
      if (!(o.sigma_grid[i] > 0)) return fail(SFW_EINVAL, "opts.sigma_grid must be > 0");
    for (int j = 0; j < o.n_d; ++j)
      if (!(o.d_grid[j] > 0)) return fail(SFW_EINVAL, "opts.d_grid must be > 0");
    if (o.max_iter < 1) return fail(SFW_EINVAL, "opts.max_iter must be >= 1");
    if (o.proposal && net_stream(o.proposal) != ws->stream)
      return fail(SFW_EINVAL, "opts.proposal must enqueue on the workspace's stream");
    S.V = (size_t)vol.nx * vol.ny * vol.nz;
    S.plan = plan_psf(ws, vol, psf);
    // graph replays of the (C, grad C) chain for this solve only
    // and autotuned launch shapes (kept in the workspace beyond the solve)
    struct GraphScope {
      sfw_workspace* ws;
      int replays0, tunings0;
      GraphScope(sfw_workspace* w, bool graphs, bool tune)
          : ws(w), replays0(w->cg_replays), tunings0(w->tune_runs) {
        ws->graphs = graphs;
        ws->tune_on = tune;
      }
      ~GraphScope() {
        ws->graphs = false;
        ws->tune_on = false;
      }
    } graph_scope(ws, o.graphs != 0, o.autotune != 0);
    const auto t0 = Clock::now();

    if (o.check_finite) {
      int* flag = reinterpret_cast<int*>(ws->best + 1);
      SFW_HIP(hipMemsetAsync(flag, 0, sizeof(int), ws->stream));
      SFW_HIP(launch_any_nonfinite(y, S.V, flag, ws->stream));
      SFW_HIP(launch_any_nonfinite(H, (size_t)psf.nx * psf.ny * psf.nz, flag, ws->stream));
      int hflag = 0;
      SFW_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, ws->stream));
      SFW_HIP(hipStreamSynchronize(ws->stream));
      if (hflag) return fail(SFW_EINVAL, "y or H holds NaN or Inf");
    }
    // direct forward operands for the LASSO columns, the PSF spectrum for the volume blur
    rc = prep_psf(ws, H, S.plan, true, !S.plan.fft);
    if (rc) return rc;
    rc = prep_spectrum(ws, H, S.plan);
    if (rc) return rc;
    // y is fixed for the whole solve: validate the LASSO column cache against it once
    rc = lasso_check_inputs(ws, S.plan, vol, y, H);
    if (rc) return rc;

    // the starting measure (mu = 0 unless the caller resumes from init_atoms)
    if (o.n_init < 0 || o.n_init > ws->max_atoms || (o.n_init > 0 && !o.init_atoms))
      return fail(SFW_EINVAL, "opts.n_init must be in [0, max_atoms] with init_atoms set");
    {
      std::vector<double> lo, hi;
      S.theta_bounds(lo, hi);
      for (int i = 0; i < o.n_init; ++i) {
        const sfw_atom& a = o.init_atoms[i];
        const double v[6] = {a.w, a.mx, a.my, a.mz, a.sigma, a.d};
        for (double x : v)
          if (!std::isfinite(x)) return fail(SFW_EINVAL, "opts.init_atoms holds NaN or Inf");
        if (v[0] < 0 || !(v[4] > 0) || !(v[5] > 0))
          return fail(SFW_EINVAL, "opts.init_atoms needs w >= 0, sigma > 0 and d > 0");
        S.atoms.push_back(v[0]);
        for (int c = 0; c < 5; ++c) S.atoms.push_back(std::min(std::max(v[1 + c], lo[c]), hi[c]));
      }
      S.prune();
      S.st.max_support = S.k();
    }

    const float T = o.trunc_T > 0 ? o.trunc_T : 12.0f;
    bool converged = false;
    bool use_net = o.proposal != nullptr;
    int it = 0;
    double C = 0.0;
    for (it = 1; it <= o.max_iter; ++it) {
      // residual of the current measure, q = Phi^T r, criterion
      rc = S.cgrad(S.atoms, C, nullptr);
      if (rc) return rc;
      // step 1: a seed (the proposal network's, else the grid maximum of eta), then local
      // ascent; a proposal whose ascent ends at eta* <= 1 + eta_tol falls back to the grid,
      // whose ascent decides. After such a rejection the grid seeds the rest of the solve:
      // the network's later maxima are then almost always atoms already found (eta = 1).
      std::vector<double> th(5);
      double eta_star = 0.0;
      bool seeded = false;
      double score = 0.0, eta_prop = 0.0;
      long long evals_prop = 0;
      if (use_net) {
        auto tp = Clock::now();
        double seed[5];
        rc = sfw_net_propose(o.proposal, ws->q, vol, (float)(1.0 / lambda), seed, &score);
        if (rc) return rc;
        S.st.n_proposals++;
        auto ta = Clock::now();
        S.st.seconds_certificate += secs(tp, ta);
        if (std::isfinite(score)) {
          th.assign(seed, seed + 5);
          rc = S.ascent(th, eta_star);
          if (rc) return rc;
          S.st.seconds_ascent += secs(ta, Clock::now());
          seeded = eta_star > 1.0 + o.eta_tol;
        }  // else no finite heatmap value: no proposal, the grid seeds
        if (!seeded) {
          S.st.n_fallbacks++;
          use_net = false;
        }
        eta_prop = eta_star;
        evals_prop = S.st.n_eval_eta;
      }
      if (!seeded) {
        auto tc = Clock::now();
        rc = op_certificate(ws, vol, ws->q, lambda, o.sigma_grid, o.n_sigma, o.d_grid, o.n_d, T,
                            nullptr);
        if (rc) return rc;
        rc = sig_wait(ws, ws->cert_sig);
        if (rc) return rc;
        const sfw_argmax best = *pinned_best(ws);
        S.st.n_certificates++;
        auto ta = Clock::now();
        S.st.seconds_certificate += secs(tc, ta);
        th = {(double)best.x, (double)best.y, (double)best.z, (double)o.sigma_grid[best.i_sigma],
              (double)o.d_grid[best.i_d]};
        rc = S.ascent(th, eta_star);
        if (rc) return rc;
        S.st.seconds_ascent += secs(ta, Clock::now());
      }
      S.st.last_eta = eta_star;
      if (o.verbose)
        std::fprintf(stderr,
                     "[sfw] k=%d C=%.9g seed=%s eta*=%.9g atoms=%d evals=%lld score=%.4g "
                     "proposal_eta*=%.6g proposal_evals=%lld\n",
                     it, C, seeded ? "proposal" : "grid", eta_star, S.k(),
                     (long long)S.st.n_eval_eta, score, eta_prop, evals_prop);
      if (eta_star <= 1.0 + o.eta_tol) {
        auto ts = Clock::now();
        if (o.mode == SFW_MODE_BSFW) {  // 2b: final slide, 3b: prune
          rc = S.slide();
          if (rc) return rc;
          S.prune();
        }

        S.st.seconds_slide += secs(ts, Clock::now());
        converged = true;
        break;
      }
      // step 2: augment the support
      if (S.k() + 1 > ws->max_atoms)
        return fail(SFW_EINVAL, "support grew beyond the workspace's max_atoms");
      S.atoms.push_back(0.0);
      S.atoms.insert(S.atoms.end(), th.begin(), th.end());
      S.st.max_support = std::max(S.st.max_support, S.k());
      // step 3: weights only
      auto tl = Clock::now();
      rc = S.lasso();
      if (rc) return rc;
      S.st.seconds_lasso += secs(tl, Clock::now());
      if (o.mode == SFW_MODE_SFW) {  // step 4: slide all parameters
        auto ts = Clock::now();
        rc = S.slide();
        if (rc) return rc;
        S.st.seconds_slide += secs(ts, Clock::now());
      }
      S.prune();  // SFW step 5 / BSFW step 4
    }
    rc = S.cgrad(S.atoms, C, nullptr);
    if (rc) return rc;
    const int n = S.k();
    S.st.iterations = converged ? it : o.max_iter;
    S.st.converged = converged ? 1 : 0;
    S.st.n_atoms = n;
    S.st.n_graph_replays = ws->cg_replays - graph_scope.replays0;
    S.st.n_tunings = ws->tune_runs - graph_scope.tunings0;
    S.st.criterion = C;
    S.st.seconds_total = secs(t0, Clock::now());
    if (stats) *stats = S.st;
    *n_out = n;
    if (n > cap) return fail(SFW_ECAP, "more atoms than cap; *n_out holds the count");
    for (int i = 0; i < n; ++i) {
      atoms_out[i].w = (float)S.atoms[6 * i + 0];
      atoms_out[i].mx = (float)S.atoms[6 * i + 1];
      atoms_out[i].my = (float)S.atoms[6 * i + 2];
      atoms_out[i].mz = (float)S.atoms[6 * i + 3];
      atoms_out[i].sigma = (float)S.atoms[6 * i + 4];
      atoms_out[i].d = (float)S.atoms[6 * i + 5];
    }
    if (!converged) return fail(SFW_ENOCONV, "iteration cap reached before eta* <= 1 + eta_tol");
    return SFW_OK;
  } catch (const std::exception& e) {
    return fail(SFW_EINVAL, std::string("exception in sfw_solve: ") + e.what());
  } catch (...) {
    return fail(SFW_EINVAL, "unexpected exception in sfw_solve");
  }
}
