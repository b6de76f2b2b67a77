// Internal operator layer shared by the C ABI (sfw_api.cpp) and the solver (sfw_solver.cpp).
#pragma once

#include <vector>

#include "sfw_internal.h"

namespace sfw {

int check_dims(const sfw_dims& d, const char* what);
int check_psf(const sfw_dims& p);
int check_ws_fit(const sfw_workspace* ws, const sfw_dims& vol, const sfw_dims* psf, int n);
int check_lambda(float lambda);

// How the PSF convolutions of one volume shape run: on the matrix cores when the PSF fits
// k_conv_mfma (pz <= 16, px * py <= 128), else on the LDS-tiled VALU kernel. The environment
// variable SFW_CONV=valu forces the VALU kernel (used by the tests to cover both).
struct PsfPlan {
  sfw_dims psf{1, 1, 1};
  ConvPlan valu;
  bool mfma = false;  // direct convolutions on the matrix cores (else the VALU kernel)
  bool fft = false;   // volume blur and adjoint through the spectrum (blur)
  BlurPlan blur;
  int nres = 0;  // number of loss partials the residual epilogue writes
};
// SFW_CONV selects the volume convolution: "fft", "mfma" or "valu" (direct kernels only);
// unset, the spectral blur is used for PSFs of at least 343 taps when the workspace holds its
// arrays.
PsfPlan plan_psf(const sfw_workspace* ws, const sfw_dims& vol, const sfw_dims& psf);
// PSF spectrum (and the plan's twiddles when its lengths changed) for a spectral plan; no-op
// otherwise.
int prep_spectrum(sfw_workspace* ws, const float* H, const PsfPlan& p);
// Build the forward (convolution) and / or adjoint (correlation) operands of H and, when atoms
// is not null, the constants of its n atoms into ws->ak, in one launch.
int prep_all(sfw_workspace* ws, const float* H, const PsfPlan& p, bool fwd, bool adj,
             const sfw_atom* atoms, int n, bool unit_weight);
int prep_psf(sfw_workspace* ws, const float* H, const PsfPlan& p, bool fwd, bool adj);
// Atom constants (see AtomK) from float64 parameters.
AtomK make_atomk(double w, double mx, double my, double mz, double sigma, double d);
// Weights-only LASSO with the workspace's column cache (see sfw_api.cpp); the cache must have
// been validated for (y, H) by lasso_check_inputs (once per y).
int lasso_check_inputs(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* y,
                       const float* H);
int op_lasso(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* y,
             const float* H, double lambda, const float* thetas, int n, std::vector<double>& w,
             bool ak_ready = false);
// out = H * in (adjoint = false) or correlation with H (adjoint = true); epilogue as launch_conv.
// Spectral when p.fft (epilogues kEpiPlain and kEpiResidual), else direct.
int conv_psf(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, bool adjoint,
             const float* in, float* out, int epi, const float* yobs, int prof_kind);
// The same on the direct kernels whatever the plan.
int conv_direct(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, bool adjoint,
                const float* in, float* out, int epi, const float* yobs, int prof_kind);
// ws->ak must hold the n atoms' constants.
int op_forward(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, int n, float* phi);
// r = y - H * f (into r_out or ws->r), q = Phi^T r (ws->q), per-atom sums and loss in sums
// (ws->dres when null; else pinned host memory, readable once ws->sums_sig has been waited
// for): sums[6a + c] (see launch_grad_finalize), sums[6n] = C, sums[6n + 1] = 1/2 ||r||^2.
int op_cgrad(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* y,
             float lambda, const sfw_atom* atoms_dev, int n, float* r_out, double* loss_out,
             sfw_atom* grad_out, double* sums = nullptr);
// q = Phi^T g (ws->q) and grad[n] = sum_s q df/d(w, m, sigma, d): the vector-Jacobian
// product of the forward model; ws->ak must hold the n atoms' constants.
int op_vjp(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* gvol,
           const sfw_atom* atoms_dev, int n, sfw_atom* grad_out);
// Tiles of the points kernel (the one-launch path, n <= kAtomArgs) that meet the cut ball of
// one of the n unit atoms hk (host constants).
GradPlan plan_points(const AtomK* hk, int n, const sfw_dims& vol);
// eta and its gradient at n points theta = (mx, my, mz, sigma, d) (host, float64); syncs.
int op_eta_points(sfw_workspace* ws, const sfw_dims& vol, const float* q, double lambda,
                  const double* thetas, int n, double* eta_out, double* grad_out);
// Grid certificate of q; the maximum lands in ws->best (device).
int op_certificate(sfw_workspace* ws, const sfw_dims& vol, const float* q, float lambda,
                   const float* sg, int ns, const float* dg, int nd, float T, float* eta_out);
// LASSO column of the unit-weight atom staged in ws->ak[atom] (parameters theta) into slot.
int op_columns(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* H, int atom,
               int slot, const float* theta);
// out[j] = <a_slot, a_(slot of j)> for j < nd, out[nd] = <a_slot, y>, float64 (device or
// pinned host memory); the slots come in sa (all of them in ws->lasso_slots when nd exceeds
// kSlotArgs).
int op_gram_row(sfw_workspace* ws, const PsfPlan& p, const sfw_dims& vol, const float* y, int slot,
                const float* theta, const SlotArgs& sa, int nd, double* out,
                const SigArgs& sig = kNoSig);
// min_{w >= 0} 1/2 w^T G w - c^T w.
int nnqp(const std::vector<double>& G, const std::vector<double>& c, int k, std::vector<double>& w);

}  // namespace sfw
