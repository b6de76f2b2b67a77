// C ABI of libsfw: workspace lifecycle, argument validation and the operator entry points.
// The solver loop (sfw_solve) lives in sfw_solver.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <new>
#include <string>

#include "sfw_internal.h"
#include "sfw_ops.h"

namespace sfw {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

const char* const kProfNames[kProfCount] = {
    "prep", "render", "conv_residual", "conv_adjoint", "conv_forward", "grad",
    "grad_finalize", "cert_conv", "cert_argmax", "lasso_render", "lasso_conv", "lasso_dots",
    "hash", "eta_grad", "cert_fft", "cert_zinv"};

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) +
                 ") in " + what;
  return SFW_EHIP;
}

// ------------------------------------------------------------------ completion signal

SigArgs sig_arm(sfw_workspace* ws) {
  if (++ws->sig_seq <= 0) ws->sig_seq = 1;  // the flag starts at 0
  return SigArgs{ws->sig_flag, ws->sig_ticket, ws->sig_seq};
}

int sig_wait(sfw_workspace* ws, const SigArgs& s) {
  if (!s.flag) {
    SFW_HIP(hipStreamSynchronize(ws->stream));
    return SFW_OK;
  }
  for (unsigned long spins = 1;; ++spins) {
    if (__atomic_load_n(s.flag, __ATOMIC_ACQUIRE) == s.seq) return SFW_OK;
    if ((spins & 0x3fff) == 0) {  // now and then: has the stream finished without the signal?
      const hipError_t e = hipStreamQuery(ws->stream);
      if (e == hipSuccess) {
        if (__atomic_load_n(s.flag, __ATOMIC_ACQUIRE) == s.seq) return SFW_OK;
        return fail(SFW_EHIP, "the stream finished without its completion signal");
      }
      if (e != hipErrorNotReady) return hip_fail(e, "waiting for a completion signal");
    }
    __builtin_ia32_pause();
  }
}

// ------------------------------------------------------------------ validation

int check_dims(const sfw_dims& d, const char* what) {
  if (d.nx <= 0 || d.ny <= 0 || d.nz <= 0)
    return fail(SFW_EINVAL, std::string(what) + ": every size must be positive");
  if ((long long)d.nx * d.ny * d.nz > (1LL << 31) - 1)
    return fail(SFW_EINVAL, std::string(what) + ": more than 2^31-1 voxels");
  return SFW_OK;
}

int check_psf(const sfw_dims& p) {
  int rc = check_dims(p, "psf");
  if (rc) return rc;
  if (p.nx % 2 == 0 || p.ny % 2 == 0 || p.nz % 2 == 0)
    return fail(SFW_EINVAL, "psf: every size must be odd (the PSF is centred at (P-1)/2)");
  return SFW_OK;
}

int check_ws_fit(const sfw_workspace* ws, const sfw_dims& vol, const sfw_dims* psf, int n) {
  if (!ws) return fail(SFW_EINVAL, "workspace is NULL");
  int rc = check_dims(vol, "vol");
  if (rc) return rc;
  if (vol.nx > ws->vol_max.nx || vol.ny > ws->vol_max.ny || vol.nz > ws->vol_max.nz)
    return fail(SFW_EINVAL, "vol exceeds the workspace's vol_max");
  if (psf) {
    rc = check_psf(*psf);
    if (rc) return rc;
    if (psf->nx > ws->psf_max.nx || psf->ny > ws->psf_max.ny || psf->nz > ws->psf_max.nz)
      return fail(SFW_EINVAL, "psf exceeds the workspace's psf_max");
  }
  if (n < 0) return fail(SFW_EINVAL, "n must be >= 0");
  if (n > ws->max_atoms) return fail(SFW_EINVAL, "n exceeds the workspace's max_atoms");
  return SFW_OK;
}

int check_lambda(float lambda) {
  if (!(lambda > 0.f) || !std::isfinite(lambda))
    return fail(SFW_EINVAL, "lambda must be finite and > 0");
  return SFW_OK;
}

// ------------------------------------------------------------------ internal operators

PsfPlan plan_psf(const sfw_workspace* ws, const sfw_dims& vol, const sfw_dims& psf) {
  PsfPlan p;
  p.psf = psf;
  p.valu = plan_conv(vol, psf.nx, psf.ny, psf.nz);
  const char* env = std::getenv("SFW_CONV");
  const bool force_valu = env && std::strcmp(env, "valu") == 0;
  const bool force_mfma = env && std::strcmp(env, "mfma") == 0;
  const bool force_fft = env && std::strcmp(env, "fft") == 0;
  p.mfma = !force_valu && mfma_conv_ok(psf.nx, psf.ny, psf.nz);
  const long long taps = (long long)psf.nx * psf.ny * psf.nz;
  if (!force_valu && !force_mfma && (force_fft || taps >= 343) && blur_plan(vol, psf, p.blur)) {
    const size_t rowp = (size_t)p.blur.px * p.blur.N[1];
    p.fft = rowp * vol.nz <= ws->blur_spec_cap && rowp * p.blur.N[2] <= ws->blur_hhat_cap;
  }
  p.nres = p.fft ? blur_residual_parts(p.blur, vol)
                 : (p.mfma ? 4 * mfma_conv_blocks(vol) : p.valu.nblocks);
  return p;
}

int prep_spectrum(sfw_workspace* ws, const float* H, const PsfPlan& p) {
  if (!p.fft) return SFW_OK;
  ProfScope ps(ws, kProfPrep);
  if (ws->blur_tw_key[0] != p.blur.N[0] || ws->blur_tw_key[1] != p.blur.N[1] ||
      ws->blur_tw_key[2] != p.blur.N[2]) {
    SFW_HIP(launch_blur_twiddles(p.blur, ws->blur_tw, ws->stream));
    for (int a = 0; a < 3; ++a) ws->blur_tw_key[a] = p.blur.N[a];
  }
  SFW_HIP(launch_psf_spectrum(p.blur, H, p.psf, ws->blur_hhat, ws->blur_hcache,
                              ws->blur_changed, ws->stream));
  return SFW_OK;
}

int prep_all(sfw_workspace* ws, const float* H, const PsfPlan& p, bool fwd, bool adj,
             const sfw_atom* atoms, int n, bool unit_weight) {
  float* of = p.mfma ? ws->am_fwd : ws->wt_fwd;
  float* oa = p.mfma ? ws->am_adj : ws->wt_adj;
  ProfScope ps(ws, kProfPrep);
  SFW_HIP(launch_prep(atoms, atoms ? n : 0, unit_weight, ws->ak, H, p.psf, p.mfma, p.valu.kzp,
                      fwd, adj, of, oa, ws->stream));
  return SFW_OK;
}

int prep_psf(sfw_workspace* ws, const float* H, const PsfPlan& p, bool fwd, bool adj) {
  return prep_all(ws, H, p, fwd, adj, nullptr, 0, false);
}

AtomK make_atomk(double w, double mx, double my, double mz, double sigma, double d) {
  AtomK k;
  k.w = (float)w;
  k.mx = (float)mx;
  k.my = (float)my;
  k.mz = (float)mz;
  k.hd = (float)(0.5 * d);
  k.hdm1 = k.hd - 1.f;
  k.c = (float)(-d * std::log2(sigma) - 1.0 + 0.52876637294489772);
  k.rcut2 = atom_rcut2(sigma, d);
  return k;
}

int conv_psf(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, bool adjoint,
             const float* in, float* out, int epi, const float* yobs, int kind) {
  if (!p.fft) return conv_direct(ws, p, vol, adjoint, in, out, epi, yobs, kind);
  if (epi != kEpiPlain && epi != kEpiResidual)
    return fail(SFW_EINVAL, "spectral blur: unsupported epilogue");
  if ((size_t)p.nres > ws->dpart_cap) return fail(SFW_EINVAL, "loss partial buffer too small");
  ProfScope ps(ws, kind);
  SFW_HIP(launch_blur(p.blur, in, vol, ws->blur_hhat, adjoint, epi, out, yobs, ws->dpart,
                      ws->blur_spec, ws->blur_tw, ws->stream));
  return SFW_OK;
}

int conv_direct(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, bool adjoint,
                const float* in, float* out, int epi, const float* yobs, int kind) {
  ProfScope ps(ws, kind);
  if (p.mfma)
    SFW_HIP(launch_conv_mfma(in, adjoint ? ws->am_adj : ws->am_fwd, p.psf, vol, epi, out, yobs,
                             ws->dpart, ws->stream));
  else
    SFW_HIP(launch_conv(p.valu, in, adjoint ? ws->wt_adj : ws->wt_fwd, vol, epi, out, yobs,
                        ws->dpart, 1.f, 0, nullptr, ws->stream));
  return SFW_OK;
}

int op_forward(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, int n, float* phi) {
  {
    ProfScope ps(ws, kProfRender, true);
    SFW_HIP(launch_render(ws->ak, n, vol, ws->f, ws->stream, kRenderVPT, ps.events()));
  }
  return conv_psf(ws, p, vol, false, ws->f, phi, kEpiPlain, nullptr, kProfConvForward);
}

// The chain of a (C, grad C) evaluation up to the per-tile gradient sums: render, blur with the
// residual and its loss partials, adjoint, gradient sums (everything but the final reduction).
static int cgrad_chain(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* y,
                       int n, float* r, const sfw_workspace::TuneChoice& shape) {
  {
    ProfScope ps(ws, kProfRender, true);
    SFW_HIP(launch_render(ws->ak, n, vol, ws->f, ws->stream, shape.render_vpt, ps.events()));
  }
  if (p.fft && p.blur.chain) {
    // residual and adjoint share the plane pass between them (see launch_blur_residual_chain)
    {
      ProfScope ps(ws, kProfConvResidual);
      SFW_HIP(launch_blur_residual_chain(p.blur, ws->f, vol, ws->blur_hhat, y, r, ws->dpart,
                                         ws->blur_spec, ws->blur_tw, ws->stream));
    }
    ProfScope ps(ws, kProfConvAdjoint);
    SFW_HIP(launch_blur_adjoint_chain(p.blur, vol, ws->blur_hhat, ws->q, ws->blur_spec,
                                      ws->blur_tw, ws->stream));
  } else {
    int rc = conv_psf(ws, p, vol, false, ws->f, r, kEpiResidual, y, kProfConvResidual);
    if (rc) return rc;
    rc = conv_psf(ws, p, vol, true, r, ws->q, kEpiPlain, nullptr, kProfConvAdjoint);
    if (rc) return rc;
  }
  ProfScope ps(ws, kProfGrad, true);
  SFW_HIP(launch_grad_items(ws->ak, n, ws->q, vol, ws->gpart, ws->gitem, shape.grad_blocks,
                            ws->stream, ps.events()));
  return SFW_OK;
}

// Enqueue the chain, or replay it from a graph (ws->graphs, no profiling): a chain whose launch
// arguments repeat those of the previous evaluation is captured into a graph, which later
// evaluations with the same arguments replay in one launch. Nothing in the chain sets memory
// with a memset; every kernel writes all it reads later.
static int cgrad_enqueue(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol,
                         const float* y, int n, float* r,
                         const sfw_workspace::TuneChoice& shape) {
  if (!ws->graphs || ws->prof_on) return cgrad_chain(ws, p, vol, y, n, r, shape);
  const std::vector<long long> key = {
      vol.nx, vol.ny, vol.nz, n, p.fft, p.blur.chain, p.mfma, p.psf.nx, p.psf.ny, p.psf.nz,
      p.blur.N[0], p.blur.N[1], p.blur.N[2], (long long)(uintptr_t)y, (long long)(uintptr_t)r,
      p.nres, shape.render_vpt, shape.grad_blocks};
  if (ws->cg_exec && key == ws->cg_key) {
    SFW_HIP(hipGraphLaunch(ws->cg_exec, ws->stream));
    ws->cg_replays++;
    return SFW_OK;
  }
  if (key != ws->cg_seen) {  // first time with these arguments: run it as it is
    ws->cg_seen = key;
    return cgrad_chain(ws, p, vol, y, n, r, shape);
  }
  if (!ws->cap_stream)
    SFW_HIP(hipStreamCreateWithFlags(&ws->cap_stream, hipStreamNonBlocking));
  hipStream_t run = ws->stream;
  ws->stream = ws->cap_stream;
  // relaxed: the sequence holds kernel launches only, and the solves of other workspaces
  // (sfw_solve_batch's threads) keep synchronising their own streams meanwhile
  hipError_t e = hipStreamBeginCapture(ws->stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    ws->stream = run;
    return hip_fail(e, "hipStreamBeginCapture");
  }
  const int rc = cgrad_chain(ws, p, vol, y, n, r, shape);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(ws->stream, &g);
  ws->stream = run;
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  if (ws->cg_exec) {
    (void)hipGraphExecDestroy(ws->cg_exec);
    ws->cg_exec = nullptr;
  }
  e = hipGraphInstantiate(&ws->cg_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    ws->cg_exec = nullptr;
    ws->cg_key.clear();
    return hip_fail(e, "hipGraphInstantiate");
  }
  ws->cg_key = key;
  ws->cg_captures++;
  SFW_HIP(hipGraphLaunch(ws->cg_exec, ws->stream));
  return SFW_OK;
}

// Launch shapes of the chain for (vol, n): the defaults, or, with ws->tune_on, the fastest of
// the candidates, timed once per (volume shape, power-of-two bucket of n) on the workspace's own
// buffers (ws->ak must hold the atoms; the render writes ws->f and the gradient sums read ws->q
// and write ws->gpart and ws->gitem, all rewritten by the evaluation that follows). The
// candidates give the same results bit for bit (the render's tiles sum every voxel's atoms in
// the same order; the gradient items are the same whatever the grid size), so the choice, which
// depends on timing, never changes a result.
static int chain_shape(sfw_workspace* ws, const sfw_dims& vol, int n,
                       sfw_workspace::TuneChoice& c) {
  c = sfw_workspace::TuneChoice();
  if (!ws->tune_on || n <= 0) return SFW_OK;
  int nb = 1;
  while (nb < n) nb <<= 1;
  const std::vector<int> key = {vol.nx, vol.ny, vol.nz, nb};
  auto it = ws->tune.find(key);
  if (it != ws->tune.end()) {
    c = it->second;
    return SFW_OK;
  }
  if (!ws->tune_ev[0]) {
    SFW_HIP(hipEventCreate(&ws->tune_ev[0]));
    SFW_HIP(hipEventCreate(&ws->tune_ev[1]));
  }
  auto timed = [&](const std::function<hipError_t()>& launch, float& best) -> int {
    best = std::numeric_limits<float>::infinity();
    for (int rep = 0; rep < 3; ++rep) {
      SFW_HIP(hipEventRecord(ws->tune_ev[0], ws->stream));
      SFW_HIP(launch());
      SFW_HIP(hipEventRecord(ws->tune_ev[1], ws->stream));
      SFW_HIP(hipEventSynchronize(ws->tune_ev[1]));
      float ms = 0.f;
      SFW_HIP(hipEventElapsedTime(&ms, ws->tune_ev[0], ws->tune_ev[1]));
      best = std::min(best, ms);
    }
    return SFW_OK;
  };
  float best_r = std::numeric_limits<float>::infinity();
  for (int vpt : {4, 8, 16}) {
    float t = 0.f;
    int rc = timed([&] { return launch_render(ws->ak, n, vol, ws->f, ws->stream, vpt); }, t);
    if (rc) return rc;
    if (t < best_r) {
      best_r = t;
      c.render_vpt = vpt;
    }
  }
  float best_g = std::numeric_limits<float>::infinity();
  for (int blocks : {1024, 2048, 4096}) {
    float t = 0.f;
    int rc = timed([&] {
      return launch_grad_items(ws->ak, n, ws->q, vol, ws->gpart, ws->gitem, blocks, ws->stream);
    }, t);
    if (rc) return rc;
    if (t < best_g) {
      best_g = t;
      c.grad_blocks = blocks;
    }
  }
  ws->tune[key] = c;
  ws->tune_runs++;
  return SFW_OK;
}

int op_cgrad(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* y,
             float lambda, const sfw_atom* atoms_dev, int n, float* r_out, double* loss_out,
             sfw_atom* grad_out, double* sums) {
  float* r = r_out ? r_out : ws->r;
  if (p.fft && p.blur.chain && (size_t)p.nres > ws->dpart_cap)
    return fail(SFW_EINVAL, "loss partial buffer too small");
  if ((size_t)grad_item_tiles(vol) * n * 6 > ws->gpart_cap)
    return fail(SFW_EINVAL, "gradient partial buffer too small");
  sfw_workspace::TuneChoice shape;
  int rc = chain_shape(ws, vol, n, shape);
  if (rc) return rc;
  rc = cgrad_enqueue(ws, p, vol, y, n, r, shape);
  if (rc) return rc;
  ws->q_valid = true;
  ProfScope ps(ws, kProfGradFinalize, true);
  // sums for the host: the finalize kernel signals them (ws->sums_sig)
  ws->sums_sig = sums ? sig_arm(ws) : kNoSig;
  SFW_HIP(launch_grad_finalize(ws->gpart, 0, ws->gitem, n, ws->dpart, p.nres, atoms_dev, lambda,
                               sums ? sums : ws->dres, grad_out, loss_out, ws->stream, false,
                               ws->sums_sig, ps.events()));
  return SFW_OK;
}

int op_vjp(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* gvol,
           const sfw_atom* atoms_dev, int n, sfw_atom* grad_out) {
  int rc = conv_psf(ws, p, vol, true, gvol, ws->q, kEpiPlain, nullptr, kProfConvAdjoint);
  if (rc) return rc;
  ws->q_valid = true;
  if (n == 0) return SFW_OK;
  if ((size_t)grad_item_tiles(vol) * n * 6 > ws->gpart_cap)
    return fail(SFW_EINVAL, "gradient partial buffer too small");
  {
    ProfScope ps(ws, kProfGrad, true);
    SFW_HIP(launch_grad_items(ws->ak, n, ws->q, vol, ws->gpart, ws->gitem,
                              sfw_workspace::TuneChoice().grad_blocks, ws->stream, ps.events()));
  }
  ProfScope ps(ws, kProfGradFinalize, true);
  SFW_HIP(launch_grad_finalize(ws->gpart, 0, ws->gitem, n, nullptr, 0, atoms_dev, 0.f, ws->dres,
                               grad_out, nullptr, ws->stream, true, kNoSig, ps.events()));
  return SFW_OK;
}

GradPlan plan_points(const AtomK* hk, int n, const sfw_dims& vol) {
  // only the tiles where some point's atom is nonzero (its cut ball) carry terms
  int box[6] = {vol.nx, 0, vol.ny, 0, vol.nz, 0};
  const int nv[3] = {vol.nx, vol.ny, vol.nz};
  for (int i = 0; i < n; ++i) {
    const double R = std::sqrt((double)hk[i].rcut2);
    const double m[3] = {hk[i].mx, hk[i].my, hk[i].mz};
    for (int a = 0; a < 3; ++a) {
      const int lo = (int)std::max(0.0, std::floor(m[a] - R));
      const int hi = (int)std::min((double)nv[a], std::ceil(m[a] + R) + 1.0);
      box[2 * a] = std::min(box[2 * a], lo);
      box[2 * a + 1] = std::max(box[2 * a + 1], hi);
    }
  }
  for (int a = 0; a < 3; ++a)
    if (box[2 * a + 1] <= box[2 * a]) {  // nothing inside the volume: one tile of zeros
      box[2 * a] = 0;
      box[2 * a + 1] = 1;
    }
  return plan_grad_box(vol, box);
}

int op_eta_points(sfw_workspace* ws, const sfw_dims& vol, const float* q, double lambda,
                  const double* thetas, int n, double* eta_out, double* grad_out) {
  // unit-weight atom constants computed on the host in float64, staged through pinned memory
  AtomK* hk = reinterpret_cast<AtomK*>(ws->hpin + ws->hp_stage);
  for (int i = 0; i < n; ++i) {
    const double* t = thetas + 5 * i;
    hk[i] = make_atomk(1.0, t[0], t[1], t[2], t[3], t[4]);
  }
  // small batches: one launch, atoms as kernel arguments, sums reduced in the kernel straight
  // into pinned host memory
  const bool one_launch = n <= kAtomArgs;
  if (!one_launch)
    SFW_HIP(hipMemcpyAsync(ws->ak, hk, sizeof(AtomK) * n, hipMemcpyHostToDevice, ws->stream));
  GradPlan gp;
  if (one_launch) gp = plan_points(hk, n, vol);
  if ((size_t)(one_launch ? gp.ntiles : grad_item_tiles(vol)) * n * 6 > ws->gpart_cap)
    return fail(SFW_EINVAL, "gradient partial buffer too small");
  double* hs = ws->hpin + ws->hp_sums;
  SigArgs sig = kNoSig;
  {
    ProfScope ps(ws, kProfEtaGrad, one_launch);  // one kernel: timed by its own events
    if (one_launch) {
      sig = sig_arm(ws);
      SFW_HIP(launch_grad_points(gp, hk, n, q, vol, ws->gpart, ws->eta_ticket, hs, sig,
                                 ws->stream, ps.events()));
    } else {
      SFW_HIP(launch_grad_items(ws->ak, n, q, vol, ws->gpart, ws->gitem,
                                sfw_workspace::TuneChoice().grad_blocks, ws->stream));
      SFW_HIP(launch_grad_finalize(ws->gpart, 0, ws->gitem, n, nullptr, 0, nullptr, 0.f,
                                   ws->dres, nullptr, nullptr, ws->stream));
    }
  }
  if (!one_launch)
    SFW_HIP(hipMemcpyAsync(hs, ws->dres, sizeof(double) * 6 * n, hipMemcpyDeviceToHost,
                           ws->stream));
  int rcw = sig_wait(ws, sig);  // kNoSig (the copy): synchronises the stream
  if (rcw) return rcw;
  const double ln2 = 0.69314718055994531;
  for (int i = 0; i < n; ++i) {
    const double* S = hs + 6 * i;
    const double* t = thetas + 5 * i;
    const double d = t[4], sg = t[3];
    eta_out[i] = S[0] / lambda;
    if (grad_out) {
      double* g = grad_out + 5 * i;
      g[0] = d * ln2 * S[3] / lambda;
      g[1] = d * ln2 * S[4] / lambda;
      g[2] = d * ln2 * S[5] / lambda;
      g[3] = (d / sg) * ln2 * S[1] / lambda;
      g[4] = -(0.5 * ln2 * ln2 * S[2] - std::log(sg) * ln2 * S[1]) / lambda;
    }
  }
  return SFW_OK;
}

static int lut_prepare(sfw_workspace* ws, const float* sg, int ns, const float* dg, int nd,
                       float T, const sfw_dims& vol) {
  std::vector<float> key;
  key.push_back(T);
  key.push_back((float)ns);
  key.push_back((float)nd);
  for (int i = 0; i < ns; ++i) key.push_back(sg[i]);
  for (int j = 0; j < nd; ++j) key.push_back(dg[j]);
  key.push_back((float)vol.nx);
  key.push_back((float)vol.ny);
  key.push_back((float)vol.nz);
  const char* fenv = std::getenv("SFW_FFT");  // transform-length policy (a test switch)
  key.push_back(fenv && std::strcmp(fenv, "generic") == 0 ? 1.f : 0.f);
  if (key == ws->lut_key && ws->lut) return SFW_OK;
  if (ns * nd > SFW_CERT_MAX_KERNELS)
    return fail(SFW_EINVAL, "n_sigma * n_d above SFW_CERT_MAX_KERNELS");
  ws->lut_key.clear();
  ws->fft_ready = false;
  std::vector<size_t> off;
  std::vector<int> rad;
  size_t total = 0;
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < nd; ++j) {
      const double R = std::ceil((double)sg[i] * std::pow(2.0 * (double)T, 1.0 / (double)dg[j]));
      const int r = (int)R;
      if (r > SFW_CERT_MAX_RADIUS)
        return fail(SFW_EINVAL, "certificate grid kernel radius above SFW_CERT_MAX_RADIUS");
      const int P = 2 * r + 1;
      ConvPlan p = plan_conv(vol, P, P, P);
      if (p.lds_bytes > (size_t)kConvMaxLds)
        return fail(SFW_EINVAL, "certificate grid kernel too wide for the convolution tile");
      off.push_back(total);
      rad.push_back(r);
      total += (size_t)P * P * p.kzp;
    }
  std::vector<float> host(total, 0.f);
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < nd; ++j) {
      const int s = i * nd + j;
      const int r = rad[s];
      const int P = 2 * r + 1;
      ConvPlan p = plan_conv(vol, P, P, P);
      const double sig = sg[i], d = dg[j];
      const double inv = 1.0 / (2.0 * std::pow(sig, d));
      float* dst = host.data() + off[s];
      for (int ky = 0; ky < P; ++ky)
        for (int kx = 0; kx < P; ++kx)
          for (int kz = 0; kz < P; ++kz) {
            const double tx = kx - r, ty = ky - r, tz = kz - r;
            const double rr = std::sqrt(tx * tx + ty * ty + tz * tz);
            dst[((size_t)ky * P + kx) * p.kzp + kz] = (float)std::exp(-std::pow(rr, d) * inv);
          }
    }
  if (total > ws->lut_cap)  // the reservation of sfw_workspace_create bounds this (no allocation)
    return fail(SFW_EINVAL, "certificate grid kernels exceed the workspace's reservation");
  SFW_HIP(hipMemcpyAsync(ws->lut, host.data(), total * sizeof(float), hipMemcpyHostToDevice,
                         ws->stream));
  SFW_HIP(hipStreamSynchronize(ws->stream));
  ws->lut_off = off;
  ws->lut_r = rad;
  // spectra of the table kernels, two per complex array
  int rmax = 0;
  for (int r : rad) rmax = std::max(rmax, r);
  FftPlan pl;
  // the Fourier-domain path runs in the arrays reserved at workspace creation; a plan that
  // does not fit them (not expected within the reservation's grid) uses the direct kernels
  const int npairs = (ns * nd + 1) / 2;
  if (fft_plan_cert(vol, rmax, pl) && (size_t)pl.px * pl.ny * pl.nz <= ws->fft_cap &&
      pl.oct <= ws->fft_oct_cap && npairs <= ws->fft_npairs_cap) {
    std::vector<float2> tw, all;
    for (int a = 0; a < 3; ++a) {
      fft_twiddles(pl.ax[a].n, tw);
      all.insert(all.end(), tw.begin(), tw.end());
    }
    // on the workspace's stream (`all` lives until the synchronisation below): nothing here
    // goes through the null stream, which another thread's solve may be capturing beside
    SFW_HIP(hipMemcpyAsync(ws->fft_tw, all.data(), all.size() * sizeof(float2),
                           hipMemcpyHostToDevice, ws->stream));
    pl.ax[0].tw = ws->fft_tw;
    pl.ax[1].tw = ws->fft_tw + pl.ax[0].n;
    pl.ax[2].tw = ws->fft_tw + pl.ax[0].n + pl.ax[1].n;
    for (int pi = 0; pi < npairs; ++pi) {
      const int sa = 2 * pi, sb = 2 * pi + 1;
      auto kz_of = [&](int s) { return plan_conv(vol, 2 * rad[s] + 1, 2 * rad[s] + 1, 2 * rad[s] + 1).kzp; };
      // full spectrum in the work array, then its octant into the dense pair table
      float2* full = ws->fft_work;
      SFW_HIP(fft_scatter_pair(pl, ws->lut + off[sa], rad[sa], kz_of(sa),
                               sb < ns * nd ? ws->lut + off[sb] : nullptr,
                               sb < ns * nd ? rad[sb] : 0, sb < ns * nd ? kz_of(sb) : 0, full,
                               ws->stream));
      SFW_HIP(fft_forward_c2c(pl, full, ws->stream));
      SFW_HIP(fft_pack_octant(pl, full, ws->fft_pairs + (size_t)pi * pl.oct, ws->stream));
    }
    SFW_HIP(hipStreamSynchronize(ws->stream));
    ws->fft = pl;
    ws->fft_ready = true;
  }
  ws->lut_key = key;
  return SFW_OK;
}

int op_certificate(sfw_workspace* ws, const sfw_dims& vol, const float* q, float lambda,
                   const float* sg, int ns, const float* dg, int nd, float T, float* eta_out) {
  int rc = lut_prepare(ws, sg, ns, dg, nd, T, vol);
  if (rc) return rc;
  const size_t V = (size_t)vol.nx * vol.ny * vol.nz;
  const char* env = std::getenv("SFW_CERT");
  const bool direct = (env && std::strcmp(env, "direct") == 0) || !ws->fft_ready;
  if (!direct) {
    const FftPlan& pl = ws->fft;
    const int nblk = fft_argmax_blocks(pl, vol);
    if ((size_t)nblk * ns * nd > ws->apart_cap)
      return fail(SFW_EINVAL, "certificate partial buffer too small");
    {
      ProfScope ps(ws, kProfCertFft);
      SFW_HIP(fft_forward_volume(pl, q, vol, ws->fft_qhat, ws->stream));
    }
    {
      ProfScope ps(ws, kProfCertZinv, true);  // timed by the kernel's own events
      SFW_HIP(fft_inverse_pairs_z(pl, ws->fft_qhat, ws->fft_pairs, ws->fft_work, ws->fft_cap,
                                  ns * nd, vol, ws->stream, ps.start(), ps.stop()));
    }
    {
      ProfScope ps(ws, kProfCertFft);
      SFW_HIP(fft_inverse_pairs_yx(pl, ws->fft_work, ws->fft_cap, ns * nd, vol, 1.0f / lambda,
                                   eta_out, ws->apart, nblk, ws->stream));
    }
    ProfScope ps(ws, kProfCertArgmax, true);
    ws->cert_sig = sig_arm(ws);
    SFW_HIP(launch_argmax_final(ws->apart, nblk * ns * nd, vol, nd, ws->best, pinned_best(ws),
                                ws->cert_sig, ws->stream, ps.events()));
    return SFW_OK;
  }
  int nb = 0;
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < nd; ++j) {
      const int s = i * nd + j;
      const int P = 2 * ws->lut_r[s] + 1;
      ConvPlan p = plan_conv(vol, P, P, P);
      nb = p.nblocks;
      if ((size_t)nb * ns * nd > ws->apart_cap)
        return fail(SFW_EINVAL, "certificate partial buffer too small");
      ProfScope ps(ws, kProfCertConv);
      SFW_HIP(launch_conv(p, q, ws->lut + ws->lut_off[s], vol, kEpiArgmax,
                          eta_out ? eta_out + (size_t)s * V : nullptr, nullptr, nullptr,
                          1.0f / lambda, (long long)s * (long long)V, ws->apart + (size_t)s * nb,
                          ws->stream));
    }
  ProfScope ps(ws, kProfCertArgmax, true);
  ws->cert_sig = sig_arm(ws);
  SFW_HIP(launch_argmax_final(ws->apart, nb * ns * nd, vol, nd, ws->best, pinned_best(ws),
                              ws->cert_sig, ws->stream, ps.events()));
  return SFW_OK;
}

// Columns a_i = H * g(theta_i) (unit weight) for i in [i0, i1) into ws->cols; atoms staged in
// ws->ak with unit weights.
static bool column_box(const float* theta, const sfw_dims& psf, const sfw_dims& vol, int box[6]);

// Column of the unit atom whose constants are ws->ak[atom] (parameters theta, host) into LASSO
// slot `slot`. Only the column's support box is computed: by the box kernel, which evaluates
// the atom itself, or after a render by the matrix-core kernel in z-chunks. The slot's box
// (ws->slot_box) records where it is valid; outside it the slot keeps whatever it held, and
// the Gram rows count the column as zero there.
int op_columns(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* H, int atom,
               int slot, const float* theta) {
  float* col = ws->cols + (size_t)slot * ws->vcap;
  int* sbox = ws->slot_box + 6 * (size_t)slot;
  int box[6];
  const bool boxed = column_box(theta, p.psf, vol, box);
  if (boxed && column_box_ok(p.psf)) {
    // the atom is computed inside the convolution kernel (no rendered volume), which also
    // records the box
    ProfScope ps(ws, kProfLassoConv);
    SFW_HIP(launch_column_box(ws->ak + atom, H, p.psf, vol, box, col, sbox, ws->stream));
    return SFW_OK;
  }
  {
    ProfScope ps(ws, kProfLassoRender);
    SFW_HIP(launch_render(ws->ak + atom, 1, vol, ws->f, ws->stream));
  }
  if (!boxed || !p.mfma) {
    const int whole[6] = {0, vol.nx, 0, vol.ny, 0, vol.nz};
    SFW_HIP(launch_store_box(whole, sbox, ws->stream));
    return conv_direct(ws, p, vol, false, ws->f, col, kEpiPlain, nullptr, kProfLassoConv);
  }
  ProfScope ps(ws, kProfLassoConv);
  SFW_HIP(launch_store_box(box, sbox, ws->stream));
  ConvRegion rg;
  rg.tx0 = box[0] / 16;
  rg.tx1 = (box[1] + 15) / 16;
  rg.ty0 = box[2] / 4;
  rg.ty1 = (box[3] + 3) / 4;
  rg.z0 = box[4];
  rg.z1 = box[5];
  // z-chunks: about two blocks per CU, at least 4 output planes each
  const int tiles = (rg.tx1 - rg.tx0) * (rg.ty1 - rg.ty0);
  const int depth = rg.z1 - rg.z0;
  const int chunks = std::max(1, std::min((512 + tiles - 1) / tiles, (depth + 3) / 4));
  rg.zchunk = (depth + chunks - 1) / chunks;
  SFW_HIP(launch_conv_mfma_region(ws->f, ws->am_fwd, p.psf, vol, rg, col, ws->stream));
  return SFW_OK;
}

// Support box of the column a = H * g of a unit atom theta = (m, sigma, d): the ball where
// u = (r / sigma)^d / 2 < kColumnCutU, of radius sigma (2 kColumnCutU)^(1/d), grown by one
// voxel and the PSF half-widths. Outside it every tap of a meets g < exp(-kColumnCutU), and the
// column is stored as zero there. x bounds are widened to multiples of 4 for vector loads.
// False when the box is the whole volume anyway.
static bool column_box(const float* theta, const sfw_dims& psf, const sfw_dims& vol, int box[6]) {
  const double sig = theta[3], d = theta[4];
  const double R = sig * std::pow(2.0 * kColumnCutU, 1.0 / d) + 1.0;
  const double c[3] = {(psf.nx - 1) / 2.0, (psf.ny - 1) / 2.0, (psf.nz - 1) / 2.0};
  const int n[3] = {vol.nx, vol.ny, vol.nz};
  bool whole = true;
  for (int a = 0; a < 3; ++a) {
    const double lo = std::floor(theta[a] - R - c[a]), hi = std::ceil(theta[a] + R + c[a]) + 1.0;
    int l = (int)std::max(0.0, std::min((double)n[a], lo));
    int h = (int)std::max(0.0, std::min((double)n[a], hi));
    if (a == 0) {
      l &= ~3;
      h = std::min(n[a], (h + 3) & ~3);
    }
    if (h <= l) {  // the column vanishes on the volume: keep a one-vector box
      l = 0;
      h = a == 0 ? std::min(4, n[a]) : 1;
    }
    box[2 * a] = l;
    box[2 * a + 1] = h;
    whole = whole && l == 0 && h == n[a];
  }
  return !whole;
}

// Gram row of slot `slot` against the nd slots sa (the first kSlotArgs; all of them in
// ws->lasso_slots when there are more), then <a, y>: out [nd + 1] (float64; device or pinned
// host memory). theta: the unit atom of the slot (host), used to restrict the sums to its
// support.
int op_gram_row(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* y, int slot,
                const float* theta, const SlotArgs& sa, int nd, double* out, const SigArgs& sig) {
  const size_t V = (size_t)vol.nx * vol.ny * vol.nz;
  const float* a = ws->cols + (size_t)slot * ws->vcap;
  ProfScope ps(ws, kProfLassoDots);
  int box[6];
  const bool boxed = column_box(theta, p.psf, vol, box);
  if (vol.nx % 4 == 0 && ws->vcap % 4 == 0 && boxed) {
    SFW_HIP(launch_dots_box(a, ws->cols, sa, ws->lasso_slots, ws->slot_box, nd, ws->vcap, y, vol,
                            box, ws->dpart, (int)std::min<size_t>(ws->dpart_cap, 1u << 30), out,
                            sig, ws->stream));
    return SFW_OK;
  }
  if (!boxed) {  // the column was computed on the whole volume
    box[0] = 0;
    box[1] = vol.nx;
    box[2] = 0;
    box[3] = vol.ny;
    box[4] = 0;
    box[5] = vol.nz;
  }
  int nb = (int)std::min<size_t>(1024, (V + 1023) / 1024);
  if ((size_t)nb * (nd + 1) > ws->dpart_cap) return fail(SFW_EINVAL, "dot partial buffer too small");
  SFW_HIP(launch_dots(a, box, ws->cols, sa, ws->lasso_slots, ws->slot_box, nd, ws->vcap, y, vol,
                      ws->dpart, nb, out, sig, ws->stream));
  return SFW_OK;
}

// Enqueue the fingerprints of y and H (and a copy of the n device atoms, if any) into the
// pinned region at hp_hash (atoms at hp_atoms); read them with read_fingerprints once *sig
// has been waited for.
static int enqueue_fingerprints(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol,
                                const float* y, const float* H, const sfw_atom* atoms, int n,
                                SigArgs* sig) {
  ProfScope ps(ws, kProfHash);
  const size_t V = (size_t)vol.nx * vol.ny * vol.nz;
  // the final kernel writes the fingerprints and the atoms straight into the pinned region,
  // then signals *sig
  *sig = sig_arm(ws);
  SFW_HIP(launch_fingerprints(y, V, H, (size_t)p.psf.nx * p.psf.ny * p.psf.nz, atoms, n,
                              ws->fp_part,
                              reinterpret_cast<unsigned long long*>(ws->hpin + ws->hp_hash),
                              reinterpret_cast<float*>(ws->hpin + ws->hp_atoms), *sig,
                              ws->stream));
  return SFW_OK;
}

static void read_fingerprints(const sfw_workspace* ws, unsigned long long* yh,
                              unsigned long long* hh) {
  const unsigned long long* fp = reinterpret_cast<const unsigned long long*>(ws->hpin + ws->hp_hash);
  *yh = fp[0];
  *hh = fp[1];
}

// Drop the cached LASSO columns unless they were computed for this y pointer, shapes,
// convolution kind and the given fingerprints of y and H.
static void lasso_validate(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol,
                           const float* y, unsigned long long yh, unsigned long long hh) {
  const bool same = ws->lasso_y == y && ws->lasso_yhash == yh && ws->lasso_hhash == hh &&
                    ws->lasso_mfma == p.mfma && ws->lasso_vol.nx == vol.nx &&
                    ws->lasso_vol.ny == vol.ny && ws->lasso_vol.nz == vol.nz &&
                    ws->lasso_psf.nx == p.psf.nx && ws->lasso_psf.ny == p.psf.ny &&
                    ws->lasso_psf.nz == p.psf.nz;
  if (!same) {
    std::fill(ws->slot_ok.begin(), ws->slot_ok.end(), 0);
    std::fill(ws->gram_ok.begin(), ws->gram_ok.end(), 0);
  }
  ws->lasso_y = y;
  ws->lasso_yhash = yh;
  ws->lasso_hhash = hh;
  ws->lasso_mfma = p.mfma;
  ws->lasso_vol = vol;
  ws->lasso_psf = p.psf;
}

// Fingerprint y and H and validate the cache (one synchronisation).
int lasso_check_inputs(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* y,
                       const float* H) {
  SigArgs sig = kNoSig;
  int rc = enqueue_fingerprints(ws, p, vol, y, H, nullptr, 0, &sig);
  if (rc) return rc;
  rc = sig_wait(ws, sig);
  if (rc) return rc;
  unsigned long long yh = 0, hh = 0;
  read_fingerprints(ws, &yh, &hh);
  lasso_validate(ws, p, vol, y, yh, hh);
  return SFW_OK;
}

// Weights-only LASSO for unit-weight atoms thetas [n][5] (host, float32 values as the device
// sees them); the PSF operands for the forward convolution must be prepared and the cache
// validated for (y, H) (lasso_check_inputs). ak_ready: the unit-weight atom constants of all n
// atoms are in ws->ak (else they are uploaded). Columns are cached in slots keyed by the atom
// parameters, and Gram entries by slot pair: only atoms without a cached column get one
// (render + blur), and only slots with a missing entry against the support get a Gram row
// (one synchronisation for the readback).
int op_lasso(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* y,
             const float* H, double lambda, const float* thetas, int n, std::vector<double>& w,
             bool ak_ready) {
  w.assign(n, 0.0);
  if (n == 0) return SFW_OK;
  const int M = ws->max_atoms;
  if (n > M) return fail(SFW_EINVAL, "LASSO support exceeds max_atoms");
  // slot of every atom: a cached column with the same parameters, else a slot no atom of this
  // support maps to (free ones first)
  std::vector<int> map(n, -1);
  std::vector<char> in_use(M, 0);
  for (int i = 0; i < n; ++i)
    for (int s2 = 0; s2 < M; ++s2)
      if (ws->slot_ok[s2] &&
          std::memcmp(&ws->slot_theta[5 * (size_t)s2], thetas + 5 * (size_t)i, 5 * sizeof(float)) == 0) {
        map[i] = s2;
        in_use[s2] = 1;
        break;
      }
  std::vector<std::pair<int, int>> fresh;  // (atom, slot)
  for (int i = 0; i < n; ++i) {
    if (map[i] >= 0) continue;
    for (int j = 0; j < i; ++j)  // a duplicate of an atom placed earlier in this call
      if (std::memcmp(thetas + 5 * (size_t)j, thetas + 5 * (size_t)i, 5 * sizeof(float)) == 0) {
        map[i] = map[j];
        break;
      }
    if (map[i] >= 0) continue;
    int slot = -1;
    for (int s2 = 0; s2 < M && slot < 0; ++s2)
      if (!ws->slot_ok[s2] && !in_use[s2]) slot = s2;
    for (int s2 = 0; s2 < M && slot < 0; ++s2)
      if (!in_use[s2]) slot = s2;
    map[i] = slot;  // n <= M guarantees a slot
    in_use[slot] = 1;
    ws->slot_ok[slot] = 0;
    for (int t = 0; t < M; ++t) ws->gram_ok[(size_t)slot * M + t] = ws->gram_ok[(size_t)t * M + slot] = 0;
    std::memcpy(&ws->slot_theta[5 * (size_t)slot], thetas + 5 * (size_t)i, 5 * sizeof(float));
    fresh.emplace_back(i, slot);
  }
  // the distinct slots of the support, in atom order
  std::vector<int> D;
  for (int i = 0; i < n; ++i)
    if (std::find(D.begin(), D.end(), map[i]) == D.end()) D.push_back(map[i]);
  const int nd = (int)D.size();
  if (!fresh.empty()) {
    if (!ak_ready) {
      AtomK* hk = reinterpret_cast<AtomK*>(ws->hpin + ws->hp_stage);
      for (int i = 0; i < n; ++i) {
        const float* t = thetas + 5 * (size_t)i;
        hk[i] = make_atomk(1.0, t[0], t[1], t[2], t[3], t[4]);
      }
      SFW_HIP(hipMemcpyAsync(ws->ak, hk, sizeof(AtomK) * n, hipMemcpyHostToDevice, ws->stream));
    }
    // columns over their support boxes go kBoxColumns at a time through one launch; the
    // others (a box covering the volume, or a PSF the box kernel does not take) one by one
    std::vector<ColumnBoxJob> jobs;
    auto flush = [&]() -> int {
      if (jobs.empty()) return SFW_OK;
      ProfScope ps(ws, kProfLassoConv, true);
      SFW_HIP(launch_column_boxes(jobs.data(), (int)jobs.size(), H, p.psf, vol, ws->stream,
                                  ps.events()));
      jobs.clear();
      return SFW_OK;
    };
    for (const auto& f : fresh) {
      ColumnBoxJob job;
      if (column_box(thetas + 5 * (size_t)f.first, p.psf, vol, job.box) && column_box_ok(p.psf)) {
        job.atom = ws->ak + f.first;
        job.out = ws->cols + (size_t)f.second * ws->vcap;
        job.box_out = ws->slot_box + 6 * (size_t)f.second;
        jobs.push_back(job);
        if ((int)jobs.size() == kBoxColumns) {
          int rc = flush();
          if (rc) return rc;
        }
      } else {
        int rc = op_columns(ws, p, vol, H, f.first, f.second, thetas + 5 * (size_t)f.first);
        if (rc) return rc;
      }
      ws->slot_ok[f.second] = 1;
    }
    int rcf = flush();
    if (rcf) return rcf;
  }
  // Gram rows for the entries missing between support slots: fresh slots first, each row
  // covering its slot's whole row and column, then any slot still missing an entry
  std::vector<int> rows;
  {
    std::vector<char> ok((size_t)nd * nd);
    for (int a = 0; a < nd; ++a)
      for (int b = 0; b < nd; ++b) ok[(size_t)a * nd + b] = ws->gram_ok[(size_t)D[a] * M + D[b]];
    std::vector<int> order;
    for (const auto& f : fresh) order.push_back((int)(std::find(D.begin(), D.end(), f.second) - D.begin()));
    for (int a = 0; a < nd; ++a)
      if (std::find(order.begin(), order.end(), a) == order.end()) order.push_back(a);
    for (int a : order) {
      bool full = true;
      for (int b = 0; b < nd && full; ++b) full = ok[(size_t)a * nd + b] != 0;
      if (full) continue;
      rows.push_back(D[a]);
      for (int b = 0; b < nd; ++b) ok[(size_t)a * nd + b] = ok[(size_t)b * nd + a] = 1;
    }
  }
  if (!rows.empty()) {
    // the slot list rides in the kernel arguments; a longer one also goes to the device
    SlotArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    std::copy(D.begin(), D.begin() + std::min(nd, kSlotArgs), sa.s);
    if (nd > kSlotArgs) {
      int* hs = reinterpret_cast<int*>(ws->hpin + ws->hp_slots);
      std::copy(D.begin(), D.end(), hs);
      SFW_HIP(hipMemcpyAsync(ws->lasso_slots, hs, sizeof(int) * nd, hipMemcpyHostToDevice,
                             ws->stream));
    }
    // the rows' final sums go straight to pinned host memory; rows over a support box go
    // kDotsRows at a time through one launch (and one final reduction), the others one by one
    const size_t stride = (size_t)nd + 1;
    double* hr = ws->hpin + ws->hp_rows;
    std::vector<char> boxed(rows.size());
    std::vector<GramRowBox> rb(rows.size());
    for (size_t r = 0; r < rows.size(); ++r) {
      rb[r].a = ws->cols + (size_t)rows[r] * ws->vcap;
      boxed[r] = vol.nx % 4 == 0 && ws->vcap % 4 == 0 &&
                 column_box(&ws->slot_theta[5 * (size_t)rows[r]], p.psf, vol, rb[r].box);
    }
    // launch groups in row order: runs of consecutive boxed rows (their sums land in
    // consecutive rows of the pinned block) whose partials fit the buffer together, and each
    // other row alone; the last group signals
    const int dcap = (int)std::min<size_t>(ws->dpart_cap, 1u << 30);
    std::vector<std::pair<size_t, size_t>> groups;  // [first, last) rows
    for (size_t r = 0; r < rows.size();) {
      size_t e = r + 1;
      if (boxed[r]) {
        size_t parts = (size_t)dots_box_blocks(rb[r].box);
        while (e < rows.size() && boxed[e] && e - r < (size_t)kDotsRows &&
               (parts + dots_box_blocks(rb[e].box)) * (size_t)(nd + 1) <= (size_t)dcap)
          parts += dots_box_blocks(rb[e++].box);
      }
      groups.emplace_back(r, e);
      r = e;
    }
    SigArgs sig = kNoSig;
    for (size_t g = 0; g < groups.size(); ++g) {
      if (g + 1 == groups.size()) sig = sig_arm(ws);
      const size_t r0 = groups[g].first, r1 = groups[g].second;
      if (boxed[r0]) {
        ProfScope ps(ws, kProfLassoDots);
        SFW_HIP(launch_dots_box_rows(rb.data() + r0, (int)(r1 - r0), ws->cols, sa,
                                     ws->lasso_slots, ws->slot_box, nd, ws->vcap, y, vol,
                                     ws->dpart, dcap, hr + r0 * stride, stride, sig, ws->stream));
      } else {
        int rc = op_gram_row(ws, p, vol, y, rows[r0], &ws->slot_theta[5 * (size_t)rows[r0]], sa,
                             nd, hr + r0 * stride, sig);
        if (rc) return rc;
      }
    }
    int rcw = sig_wait(ws, sig);
    if (rcw) return rcw;
    for (size_t r = 0; r < rows.size(); ++r) {
      const int sa = rows[r];
      const double* row = hr + r * stride;
      for (int b = 0; b < nd; ++b) {
        const int sb = D[b];
        ws->lasso_G[(size_t)sa * M + sb] = ws->lasso_G[(size_t)sb * M + sa] = row[b];
        ws->gram_ok[(size_t)sa * M + sb] = ws->gram_ok[(size_t)sb * M + sa] = 1;
      }
      ws->lasso_b[sa] = row[nd];
    }
  }
  std::vector<double> Gk((size_t)n * n), c(n);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) Gk[(size_t)i * n + j] = ws->lasso_G[(size_t)map[i] * M + map[j]];
    c[i] = ws->lasso_b[map[i]] - lambda;
  }
  return nnqp(Gk, c, n, w);
}

}  // namespace sfw

using namespace sfw;

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* sfw_last_error(void) { return g_last_error.c_str(); }

int sfw_default_options(sfw_options* o) {
  if (!o) return fail(SFW_EINVAL, "opts is NULL");
  std::memset(o, 0, sizeof(*o));
  o->mode = SFW_MODE_BSFW;
  o->n_sigma = 4;
  for (int i = 0; i < 4; ++i) o->sigma_grid[i] = 1.0f + i / 3.0f;
  o->n_d = 3;
  o->d_grid[0] = 1.5f;
  o->d_grid[1] = 2.0f;
  o->d_grid[2] = 2.5f;
  o->sigma_lo = 0.5f;
  o->sigma_hi = 4.0f;
  o->d_lo = 1.2f;
  o->d_hi = 3.0f;
  o->trunc_T = 12.0f;
  o->eta_tol = 1e-3;
  o->prune_rel = 1e-6;
  o->merge_tol = 5e-2;
  o->max_iter = 200;
  o->ascent_max_iter = 200;
  o->slide_max_iter = 1000;
  o->ascent_gtol = 1e-9;
  o->slide_gtol = 1e-9;
  o->ftol = 1e-12;
  o->lbfgs_memory = 40;
  o->check_finite = 1;
  o->verbose = 0;
  o->slide_slope_tol = 1e-6;
  o->graphs = 0;
  o->autotune = 1;
  return SFW_OK;
}

void sfw_workspace_destroy(sfw_workspace* ws) {
  if (!ws) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(ws->device);
  if (ws->stream) (void)hipStreamSynchronize(ws->stream);
  if (ws->cg_exec) (void)hipGraphExecDestroy(ws->cg_exec);
  if (ws->cap_stream) (void)hipStreamDestroy(ws->cap_stream);
  for (hipEvent_t e : ws->tune_ev)
    if (e) (void)hipEventDestroy(e);
  float* fbufs[] = {ws->f, ws->phi, ws->r, ws->q, ws->tmpv, ws->wt_fwd, ws->wt_adj, ws->am_fwd,
                    ws->am_adj, ws->lut, ws->gpart, ws->cols};
  for (float* b : fbufs)
    if (b) (void)hipFree(b);
  if (ws->atoms_dev) (void)hipFree(ws->atoms_dev);
  if (ws->ak) (void)hipFree(ws->ak);
  if (ws->dpart) (void)hipFree(ws->dpart);
  if (ws->dres) (void)hipFree(ws->dres);
  if (ws->apart) (void)hipFree(ws->apart);
  if (ws->best) (void)hipFree(ws->best);
  if (ws->lasso_slots) (void)hipFree(ws->lasso_slots);
  if (ws->fft_tw) (void)hipFree(ws->fft_tw);
  if (ws->fft_qhat) (void)hipFree(ws->fft_qhat);
  if (ws->fft_work) (void)hipFree(ws->fft_work);
  if (ws->fft_pairs) (void)hipFree(ws->fft_pairs);
  if (ws->blur_spec) (void)hipFree(ws->blur_spec);
  if (ws->blur_hhat) (void)hipFree(ws->blur_hhat);
  if (ws->blur_tw) (void)hipFree(ws->blur_tw);
  if (ws->blur_hcache) (void)hipFree(ws->blur_hcache);
  if (ws->blur_changed) (void)hipFree(ws->blur_changed);
  if (ws->eta_ticket) (void)hipFree(ws->eta_ticket);
  if (ws->gitem) (void)hipFree(ws->gitem);
  if (ws->hpin) (void)hipHostFree(ws->hpin);
  if (ws->sig_flag) (void)hipHostFree(ws->sig_flag);
  if (ws->sig_ticket) (void)hipFree(ws->sig_ticket);
  if (ws->fp_part) (void)hipFree(ws->fp_part);
  if (ws->slot_box) (void)hipFree(ws->slot_box);
  for (hipEvent_t e : ws->prof_start) (void)hipEventDestroy(e);
  for (hipEvent_t e : ws->prof_stop) (void)hipEventDestroy(e);
  (void)hipSetDevice(cur);
  delete ws;
}

int sfw_workspace_create(sfw_workspace** out, sfw_dims vol_max, sfw_dims psf_max, int max_atoms,
                         hipStream_t stream) {
  try {
    if (!out) return fail(SFW_EINVAL, "ws output pointer is NULL");
    *out = nullptr;
    int rc = check_dims(vol_max, "vol_max");
    if (rc) return rc;
    rc = check_psf(psf_max);
    if (rc) return rc;
    if (max_atoms < 1 || max_atoms > 4096)
      return fail(SFW_EINVAL, "max_atoms must be in [1, 4096]");
    {
      // PSF must fit the convolution's LDS tile even with one y tap per pass
      const int LX = kConvTX + psf_max.nx - 1;
      if ((size_t)LX * kConvTY * conv_tile_lzp(4) * 4 > (size_t)kConvMaxLds)
        return fail(SFW_EINVAL, "psf_max.nx too large for the convolution tile");
    }
    sfw_workspace* ws = new (std::nothrow) sfw_workspace();
    if (!ws) return fail(SFW_ENOMEM, "host allocation failed");
    SFW_HIP(hipGetDevice(&ws->device));
    ws->stream = stream;
    ws->vol_max = vol_max;
    ws->psf_max = psf_max;
    ws->max_atoms = max_atoms;
    // volume capacity in elements, a multiple of 64 (aligned columns for vector loads)
    ws->vcap = ((size_t)vol_max.nx * vol_max.ny * vol_max.nz + 63) / 64 * 64;
    const size_t V = ws->vcap;
    const int na = max_atoms + 1;
    auto dmalloc = [&](void** p, size_t bytes, const char* what) -> int {
      hipError_t e = hipMalloc(p, bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SFW_ENOMEM, std::string("device allocation failed: ") + what);
      }
      return SFW_OK;
    };
#define ALLOC(ptr, bytes, what)                                    \
  do {                                                             \
    int rc_ = dmalloc(reinterpret_cast<void**>(&(ptr)), (bytes), what); \
    if (rc_) {                                                     \
      sfw_workspace_destroy(ws);                                   \
      return rc_;                                                  \
    }                                                              \
  } while (0)
    ALLOC(ws->f, V * 4, "f");
    ALLOC(ws->phi, V * 4, "phi");
    ALLOC(ws->r, V * 4, "r");
    ALLOC(ws->q, V * 4, "q");
    ALLOC(ws->tmpv, V * 4, "tmpv");
    ws->wt_cap = (size_t)psf_max.nx * psf_max.ny * (psf_max.nz + 15);
    ALLOC(ws->wt_fwd, ws->wt_cap * 4, "psf copy");
    ALLOC(ws->wt_adj, ws->wt_cap * 4, "psf copy");
    ALLOC(ws->am_fwd, 32 * 64 * 4, "psf matrix operands");
    ALLOC(ws->am_adj, 32 * 64 * 4, "psf matrix operands");
    ALLOC(ws->atoms_dev, sizeof(sfw_atom) * na, "atoms");
    ALLOC(ws->ak, sizeof(AtomK) * na, "atom constants");
    const size_t nxy = (size_t)vol_max.nx * vol_max.ny;
    // gradient tiles: 16 x 16 (y, x) patches times z chunks of at least 16 planes
    const size_t gtiles = (size_t)((vol_max.nx + 15) / 16) * ((vol_max.ny + 15) / 16) *
                          ((vol_max.nz + 15) / 16);
    ws->gpart_cap = gtiles * na * 6;
    ALLOC(ws->gpart, ws->gpart_cap * 4, "gradient partials");
    ALLOC(ws->gitem, sizeof(int) * (na + 1), "gradient item offsets");
    const size_t cblocks = (size_t)((vol_max.nx + kConvTX - 1) / kConvTX) *
                           ((vol_max.ny + kConvTY - 1) / kConvTY) *
                           ((vol_max.nz + kConvRZ - 1) / kConvRZ);
    const size_t mparts = 4 * (size_t)mfma_conv_blocks(vol_max);
    const size_t bparts = (size_t)((vol_max.ny + 15) / 16) * vol_max.nz;  // spectral residual
    ws->dpart_cap = std::max(std::max(std::max(cblocks, mparts), bparts), (size_t)1024 * (na + 2));
    ALLOC(ws->dpart, ws->dpart_cap * 8, "float64 partials");
    const size_t dres_n = (size_t)(na + 2) * (na + 2) + 8 * (size_t)(na + 2) + 64;
    ALLOC(ws->dres, dres_n * 8, "float64 results");
    // argmax partials: per table kernel, the blocks of a direct certificate convolution or of
    // the last Fourier pass (at least 8 lines of one plane per block)
    const size_t fblocks = (size_t)((vol_max.ny + 7) / 8) * vol_max.nz;
    ws->apart_cap = std::max(cblocks, fblocks) * SFW_MAX_GRID * SFW_MAX_GRID;
    ALLOC(ws->apart, ws->apart_cap * sizeof(ArgPart), "argmax partials");
    ALLOC(ws->best, sizeof(sfw_argmax) * 2, "argmax");
    ALLOC(ws->cols, (size_t)max_atoms * V * 4, "LASSO columns");
    {
      // spectral blur arrays for the largest plan (lengths grow with the volume and the PSF;
      // axes past kFftMaxBlur use the direct kernels)
      const int nmax[3] = {vol_max.nx, vol_max.ny, vol_max.nz};
      const int cmax[3] = {(psf_max.nx - 1) / 2, (psf_max.ny - 1) / 2, (psf_max.nz - 1) / 2};
      int L[3];
      for (int a = 0; a < 3; ++a) {
        L[a] = kFftMaxBlur;
        int r1 = 0, r2 = 0;
        for (int m = std::max(nmax[a] + cmax[a], 16); m <= kFftMaxBlur; ++m)
          if (fft_fixed_plan(m, &r1, &r2)) {
            L[a] = m;
            break;
          }
      }
      // planes may take the longer of the two in-plane lengths for both axes (blur_plan)
      const int Lp = std::max(L[0], L[1]);
      const size_t px = (size_t)((Lp / 2 + 1 + 3) & ~3);
      ws->blur_spec_cap = px * Lp * vol_max.nz;
      ws->blur_hhat_cap = px * Lp * L[2];
      ALLOC(ws->blur_spec, ws->blur_spec_cap * sizeof(float2), "blur spectrum");
      ALLOC(ws->blur_hhat, ws->blur_hhat_cap * sizeof(float2), "PSF spectrum");
      ALLOC(ws->blur_tw, 3 * (size_t)kFftMaxBlur * sizeof(float2), "blur twiddles");
      ALLOC(ws->blur_hcache, (size_t)kHcacheFloats * sizeof(float), "PSF spectrum key");
      ALLOC(ws->blur_changed, sizeof(int), "PSF spectrum flag");
      ALLOC(ws->eta_ticket, sizeof(int), "eta block counter");
      if (hipMemset(ws->eta_ticket, 0, sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        sfw_workspace_destroy(ws);
        return fail(SFW_EHIP, "clearing the eta block counter failed");
      }
      if (hipMemset(ws->blur_hcache, 0, (size_t)kHcacheFloats * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        sfw_workspace_destroy(ws);
        return fail(SFW_EHIP, "clearing the PSF spectrum key failed");
      }
    }
    {
      // grid certificate: the table kernels of up to SFW_CERT_MAX_KERNELS grid points of radius
      // up to SFW_CERT_MAX_RADIUS, and the Fourier-domain arrays of their largest plan at
      // vol_max, so that sfw_certificate allocates nothing
      const int P = 2 * SFW_CERT_MAX_RADIUS + 1;
      ws->lut_cap = (size_t)SFW_CERT_MAX_KERNELS * P * P * plan_conv(vol_max, P, P, P).kzp;
      ALLOC(ws->lut, ws->lut_cap * sizeof(float), "certificate table kernels");
      FftPlan pl;
      if (fft_plan_cert(vol_max, SFW_CERT_MAX_RADIUS, pl)) {
        ws->fft_cap = (size_t)pl.px * pl.ny * pl.nz;
        ws->fft_oct_cap = pl.oct;
        ws->fft_npairs_cap = (SFW_CERT_MAX_KERNELS + 1) / 2;
        ALLOC(ws->fft_qhat, ws->fft_cap * sizeof(float2), "certificate spectrum");
        ALLOC(ws->fft_work, ws->fft_npairs_cap * ws->fft_cap * sizeof(float2),
              "certificate work arrays");
        ALLOC(ws->fft_pairs, ws->fft_npairs_cap * ws->fft_oct_cap * sizeof(float2),
              "certificate pair spectra");
        ALLOC(ws->fft_tw, 3 * (size_t)kFftMaxLen * sizeof(float2), "certificate twiddles");
      }
    }
    ALLOC(ws->lasso_slots, (size_t)max_atoms * sizeof(int), "LASSO slot list");
    ALLOC(ws->sig_ticket, sizeof(unsigned), "completion signal counter");
    ALLOC(ws->fp_part, 2 * (size_t)kFpParts * sizeof(unsigned long long), "fingerprint partials");
    ALLOC(ws->slot_box, 6 * (size_t)max_atoms * sizeof(int), "LASSO column boxes");
    if (hipMemset(ws->sig_ticket, 0, sizeof(unsigned)) != hipSuccess) {
      (void)hipGetLastError();
      sfw_workspace_destroy(ws);
      return fail(SFW_EHIP, "clearing the completion signal counter failed");
    }
    ws->slot_theta.assign(5 * (size_t)max_atoms, 0.f);
    ws->slot_ok.assign((size_t)max_atoms, 0);
    ws->gram_ok.assign((size_t)max_atoms * max_atoms, 0);
    ws->lasso_G.assign((size_t)max_atoms * max_atoms, 0.0);
    ws->lasso_b.assign((size_t)max_atoms, 0.0);
#undef ALLOC
    ws->hp_hash = 0;
    ws->hp_atoms = ws->hp_hash + 2;  // right behind the two fingerprints
    ws->hp_stage = ws->hp_atoms + 3 * (size_t)na;
    ws->hp_sums = ws->hp_stage + 4 * (size_t)na;
    ws->hp_rows = ws->hp_sums + 6 * (size_t)na + 8;
    ws->hp_slots = ws->hp_rows + (size_t)(na + 2) * (na + 2) + 64;
    ws->hp_best = ws->hp_slots + (size_t)na / 2 + 8;
    ws->hpin_cap = ws->hp_best + 4;
    if (hipHostMalloc(reinterpret_cast<void**>(&ws->hpin), ws->hpin_cap * 8, 0) != hipSuccess) {
      (void)hipGetLastError();
      sfw_workspace_destroy(ws);
      return fail(SFW_ENOMEM, "pinned host allocation failed");
    }
    // the completion flag: coherent, so that the kernels' stores reach host memory directly
    if (hipHostMalloc(reinterpret_cast<void**>(&ws->sig_flag), 64, hipHostMallocCoherent) !=
        hipSuccess) {
      (void)hipGetLastError();
      sfw_workspace_destroy(ws);
      return fail(SFW_ENOMEM, "pinned host allocation of the completion flag failed");
    }
    *ws->sig_flag = 0;
    *out = ws;
    return SFW_OK;
  } catch (const std::exception& e) {
    return fail(SFW_ENOMEM, std::string("exception: ") + e.what());
  } catch (...) {
    return fail(SFW_ENOMEM, "unknown exception");
  }
}

int sfw_profile_begin(sfw_workspace* ws, const char* classes) {
  if (!ws) return fail(SFW_EINVAL, "workspace is NULL");
  unsigned mask = 0;
  if (!classes || !*classes) {
    mask = (1u << kProfCount) - 1u;
  } else {
    std::string list(classes);
    size_t a = 0;
    while (a <= list.size()) {
      size_t b = list.find(',', a);
      if (b == std::string::npos) b = list.size();
      const std::string name = list.substr(a, b - a);
      int k = 0;
      while (k < kProfCount && name != kProfNames[k]) ++k;
      if (k == kProfCount) return fail(SFW_EINVAL, "unknown profile class '" + name + "'");
      mask |= 1u << k;
      a = b + 1;
    }
  }
  if (ws->prof_start.empty()) {
    ws->prof_start.resize(kProfPool);
    ws->prof_stop.resize(kProfPool);
    ws->prof_kind.resize(kProfPool);
    for (int i = 0; i < kProfPool; ++i) {
      SFW_HIP(hipEventCreate(&ws->prof_start[i]));
      SFW_HIP(hipEventCreate(&ws->prof_stop[i]));
    }
  }
  ws->prof_used = 0;
  ws->prof_overflow = false;
  ws->prof_mask = mask;
  ws->prof_on = true;
  return SFW_OK;
}

int sfw_profile_end(sfw_workspace* ws, sfw_prof_entry* out, int* n_out) {
  if (!ws || !out || !n_out) return fail(SFW_EINVAL, "ws, out or n_out is NULL");
  ws->prof_on = false;
  SFW_HIP(hipStreamSynchronize(ws->stream));
  double ms[kProfCount] = {0};
  int cnt[kProfCount] = {0};
  for (int i = 0; i < ws->prof_used; ++i) {
    float t = 0.f;
    SFW_HIP(hipEventElapsedTime(&t, ws->prof_start[i], ws->prof_stop[i]));
    ms[ws->prof_kind[i]] += t;
    cnt[ws->prof_kind[i]]++;
  }
  int k = 0;
  for (int i = 0; i < kProfCount && k < SFW_PROF_KINDS; ++i) {
    if (!cnt[i]) continue;
    std::memset(&out[k], 0, sizeof(out[k]));
    std::strncpy(out[k].name, kProfNames[i], sizeof(out[k].name) - 1);
    out[k].launches = cnt[i];
    out[k].ms = ms[i];
    ++k;
  }
  *n_out = k;
  if (ws->prof_overflow) return fail(SFW_EINVAL, "profile event pool exhausted; totals partial");
  return SFW_OK;
}

int sfw_workspace_set_stream(sfw_workspace* ws, hipStream_t stream) {
  if (!ws) return fail(SFW_EINVAL, "workspace is NULL");
  ws->stream = stream;
  return SFW_OK;
}

int sfw_forward(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol,
                const sfw_atom* atoms, int n, float* phi_mu) {
  try {
    int rc = check_ws_fit(ws, vol, &psf, n);
    if (rc) return rc;
    if (!H) return fail(SFW_EINVAL, "H is NULL");
    if (n > 0 && !atoms) return fail(SFW_EINVAL, "atoms is NULL");
    PsfPlan p = plan_psf(ws, vol, psf);
    rc = prep_all(ws, H, p, !p.fft, false, atoms, n, false);
    if (rc) return rc;
    rc = prep_spectrum(ws, H, p);
    if (rc) return rc;
    return op_forward(ws, p, vol, n, phi_mu ? phi_mu : ws->phi);
  } catch (...) {
    return fail(SFW_EINVAL, "unexpected exception in sfw_forward");
  }
}

int sfw_residual_grad(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol,
                      const float* y, float lambda, const sfw_atom* atoms, int n, float* r_out,
                      double* loss_out, sfw_atom* grad_out) {
  try {
    int rc = check_ws_fit(ws, vol, &psf, n);
    if (rc) return rc;
    if (!H || !y) return fail(SFW_EINVAL, "H or y is NULL");
    if (n > 0 && !atoms) return fail(SFW_EINVAL, "atoms is NULL");
    rc = check_lambda(lambda);
    if (rc) return rc;
    PsfPlan p = plan_psf(ws, vol, psf);
    rc = prep_all(ws, H, p, !p.fft, !p.fft, atoms, n, false);
    if (rc) return rc;
    rc = prep_spectrum(ws, H, p);
    if (rc) return rc;
    return op_cgrad(ws, p, vol, y, lambda, atoms, n, r_out, loss_out, n > 0 ? grad_out : nullptr);
  } catch (...) {
    return fail(SFW_EINVAL, "unexpected exception in sfw_residual_grad");
  }
}

int sfw_adjoint(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol, const float* r,
                float* q_out) {
  try {
    int rc = check_ws_fit(ws, vol, &psf, 0);
    if (rc) return rc;
    if (!H || !r || !q_out) return fail(SFW_EINVAL, "H, r or q_out is NULL");
    PsfPlan p = plan_psf(ws, vol, psf);
    rc = prep_psf(ws, H, p, false, !p.fft);
    if (rc) return rc;
    rc = prep_spectrum(ws, H, p);
    if (rc) return rc;
    return conv_psf(ws, p, vol, true, r, q_out, kEpiPlain, nullptr, kProfConvAdjoint);
  } catch (...) {
    return fail(SFW_EINVAL, "unexpected exception in sfw_adjoint");
  }
}

int sfw_forward_vjp(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol,
                    const float* g, const sfw_atom* atoms, int n, sfw_atom* grad_out) {
  try {
    int rc = check_ws_fit(ws, vol, &psf, n);
    if (rc) return rc;
    if (!H || !g) return fail(SFW_EINVAL, "H or g is NULL");
    if (n > 0 && (!atoms || !grad_out)) return fail(SFW_EINVAL, "atoms or grad_out is NULL");
    PsfPlan p = plan_psf(ws, vol, psf);
    rc = prep_all(ws, H, p, false, !p.fft, atoms, n, false);
    if (rc) return rc;
    rc = prep_spectrum(ws, H, p);
    if (rc) return rc;
    return op_vjp(ws, p, vol, g, atoms, n, grad_out);
  } catch (...) {
    return fail(SFW_EINVAL, "unexpected exception in sfw_forward_vjp");
  }
}

int sfw_certificate(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol, const float* r,
                    float lambda, const float* sigma_grid, int ns, const float* d_grid, int nd,
                    float trunc_T, float* eta_out, sfw_argmax* best_out) {
  try {
    int rc = check_ws_fit(ws, vol, &psf, 0);
    if (rc) return rc;
    if (!H) return fail(SFW_EINVAL, "H is NULL");
    if (!r && !ws->q_valid) return fail(SFW_EINVAL, "r is NULL and no q was computed yet");
    rc = check_lambda(lambda);
    if (rc) return rc;
    if (!sigma_grid || !d_grid) return fail(SFW_EINVAL, "sigma_grid or d_grid is NULL");
    if (ns < 1 || nd < 1 || ns > SFW_MAX_GRID || nd > SFW_MAX_GRID)
      return fail(SFW_EINVAL, "grid sizes must be in [1, SFW_MAX_GRID]");
    for (int i = 0; i < ns; ++i)
      if (!(sigma_grid[i] > 0.f) || !std::isfinite(sigma_grid[i]))
        return fail(SFW_EINVAL, "sigma_grid values must be finite and > 0");
    for (int j = 0; j < nd; ++j)
      if (!(d_grid[j] > 0.f) || !std::isfinite(d_grid[j]))
        return fail(SFW_EINVAL, "d_grid values must be finite and > 0");
    const float T = trunc_T > 0.f ? trunc_T : 12.0f;
    if (r) {
      PsfPlan p = plan_psf(ws, vol, psf);
      rc = prep_psf(ws, H, p, false, !p.fft);
      if (rc) return rc;
      rc = prep_spectrum(ws, H, p);
      if (rc) return rc;
      rc = conv_psf(ws, p, vol, true, r, ws->q, kEpiPlain, nullptr, kProfConvAdjoint);
      if (rc) return rc;
      ws->q_valid = true;
    }
    rc = op_certificate(ws, vol, ws->q, lambda, sigma_grid, ns, d_grid, nd, T, eta_out);
    if (rc) return rc;
    if (best_out) {
      hipPointerAttribute_t attr;
      const bool on_device = hipPointerGetAttributes(&attr, best_out) == hipSuccess &&
                             attr.type == hipMemoryTypeDevice;
      if (!on_device) (void)hipGetLastError();
      if (on_device) {
        SFW_HIP(hipMemcpyAsync(best_out, ws->best, sizeof(sfw_argmax), hipMemcpyDeviceToDevice,
                               ws->stream));
      } else {
        // the final kernel also wrote the maximum to pinned host memory, then signalled
        rc = sig_wait(ws, ws->cert_sig);
        if (rc) return rc;
        *best_out = *pinned_best(ws);
      }
    }
    return SFW_OK;
  } catch (...) {
    return fail(SFW_EINVAL, "unexpected exception in sfw_certificate");
  }
}

int sfw_eta_points(sfw_workspace* ws, sfw_dims vol, const float* q, float lambda,
                   const float* thetas, int n, double* eta_out, double* grad_out) {
  try {
    int rc = check_ws_fit(ws, vol, nullptr, n);
    if (rc) return rc;
    rc = check_lambda(lambda);
    if (rc) return rc;
    if (n == 0) return SFW_OK;
    if (!thetas || !eta_out) return fail(SFW_EINVAL, "thetas or eta_out is NULL");
    if (!q && !ws->q_valid) return fail(SFW_EINVAL, "no q given and none computed yet");
    std::vector<double> th(5 * (size_t)n);
    for (int i = 0; i < n; ++i) {
      for (int c = 0; c < 5; ++c) th[5 * i + c] = thetas[5 * i + c];
      if (!(th[5 * i + 3] > 0) || !(th[5 * i + 4] > 0))
        return fail(SFW_EINVAL, "sigma and d must be > 0");
    }
    return op_eta_points(ws, vol, q ? q : ws->q, lambda, th.data(), n, eta_out, grad_out);
  } catch (...) {
    return fail(SFW_EINVAL, "unexpected exception in sfw_eta_points");
  }
}

int sfw_lasso_weights(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol,
                      const float* y, float lambda, const sfw_atom* atoms, int n, double* w_out) {
  try {
    int rc = check_ws_fit(ws, vol, &psf, n);
    if (rc) return rc;
    if (!H || !y) return fail(SFW_EINVAL, "H or y is NULL");
    rc = check_lambda(lambda);
    if (rc) return rc;
    if (n == 0) return SFW_OK;
    if (!atoms || !w_out) return fail(SFW_EINVAL, "atoms or w_out is NULL");
    PsfPlan p = plan_psf(ws, vol, psf);
    // PSF operands (the columns use the direct kernels) and the unit-weight constants of every
    // atom, from the device atoms
    rc = prep_all(ws, H, p, true, false, atoms, n, true);
    if (rc) return rc;
    // one synchronisation brings back the atoms and the fingerprints of y and H
    SigArgs sig = kNoSig;
    rc = enqueue_fingerprints(ws, p, vol, y, H, atoms, n, &sig);
    if (rc) return rc;
    rc = sig_wait(ws, sig);
    if (rc) return rc;
    unsigned long long yh = 0, hh = 0;
    read_fingerprints(ws, &yh, &hh);
    lasso_validate(ws, p, vol, y, yh, hh);
    const sfw_atom* ha = reinterpret_cast<const sfw_atom*>(ws->hpin + ws->hp_atoms);
    std::vector<float> th(5 * (size_t)n);
    for (int i = 0; i < n; ++i) {
      th[5 * i + 0] = ha[i].mx;
      th[5 * i + 1] = ha[i].my;
      th[5 * i + 2] = ha[i].mz;
      th[5 * i + 3] = ha[i].sigma;
      th[5 * i + 4] = ha[i].d;
      if (!(ha[i].sigma > 0.f) || !(ha[i].d > 0.f))
        return fail(SFW_EINVAL, "atoms: sigma and d must be > 0");
    }
    std::vector<double> w;
    rc = op_lasso(ws, p, vol, y, H, lambda, th.data(), n, w, true);
    if (rc) return rc;
    // stream-ordered store; the values travel in the kernel arguments
    SFW_HIP(launch_store_doubles(w.data(), n, w_out, ws->stream));
    return SFW_OK;
  } catch (...) {
    return fail(SFW_EINVAL, "unexpected exception in sfw_lasso_weights");
  }
}

}  // extern "C"
