/*
 * sfw.h -- C ABI of the MI355X (gfx950) hot path of the boosted Sliding
 * Frank-Wolfe solver for gridless 3D deconvolution (Courbot & Colicchio,
 * "Boosting the Sliding Frank-Wolfe solver for 3D deconvolution",
 * arXiv:2009.05473).
 *
 * Problem (section 1.1): y = H * sum_n G(theta_n, w_n) + eps with atoms
 *   G(theta, w; s) = w exp(-||m - s||^d / (2 sigma^d)),  theta = (m, sigma, d),
 * and the criterion (section 1.2)
 *   C(y, mu, lambda) = 1/2 ||y - Phi mu||^2 + lambda sum_n w_n.
 *
 * Conventions shared by every entry point:
 *   - A volume is float32, C order [nz][ny][nx] (x fastest); voxel centres
 *     sit at integer coordinates with unit spacing on every axis.
 *   - The PSF H is float32 [pz][py][px], every size odd, centred at
 *     ((px-1)/2, (py-1)/2, (pz-1)/2). The library never normalises it.
 *   - H * f is the zero-padded linear convolution whose output lies on the
 *     volume grid; Phi^T is its exact adjoint (correlation with H).
 *   - An atom is sfw_atom (w, mx, my, mz, sigma, d) in voxel units; the
 *     gradient of C uses the same struct, each field holding dC/d(field).
 *   - Unless stated otherwise every pointer is DEVICE memory owned by the
 *     caller. The library never frees caller memory.
 *   - Operator calls enqueue on the workspace stream and return without a
 *     host synchronisation; the caller keeps inputs alive until the stream
 *     reaches that point. sfw_lasso_weights and sfw_solve synchronise.
 *   - Every call returns an int status (SFW_OK or a negative SFW_E* code).
 *     On error, sfw_last_error() returns a message for the calling thread.
 *     No C++ exception crosses this interface. Calls that share a workspace
 *     must not overlap; distinct workspaces are independent.
 */
#ifndef SFW_H
#define SFW_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SFW_OK = 0,
  SFW_EINVAL = -1,  /* invalid argument: null required pointer, dims <= 0, even PSF dims,
                       lambda <= 0 or not finite, n < 0, n > max_atoms, sizes above the
                       workspace maxima, sigma <= 0 or d <= 0, non-finite y or H (sfw_solve) */
  SFW_ENOMEM = -2,  /* device or host allocation failed (workspace creation only) */
  SFW_EHIP = -3,    /* a HIP runtime call failed; the message names it */
  SFW_ECAP = -4,    /* sfw_solve: more atoms than cap; *n_out holds the needed size */
  SFW_ENOCONV = -5  /* sfw_solve: iteration cap reached; best measure so far is returned */
};

enum { SFW_MODE_BSFW = 0, SFW_MODE_SFW = 1 };

#define SFW_MAX_GRID 16
/* A workspace reserves the grid certificate (its table kernels and Fourier-domain arrays) at
 * creation for up to SFW_CERT_MAX_KERNELS grid points (n_sigma * n_d) whose kernels reach
 * radius R = ceil(sigma (2T)^(1/d)) <= SFW_CERT_MAX_RADIUS (e.g. sigma <= 4.8 at d = 1.5,
 * T = 12), so that sfw_certificate and sfw_solve allocate nothing; larger grids are rejected. */
#define SFW_CERT_MAX_KERNELS 16
#define SFW_CERT_MAX_RADIUS 40

typedef struct { int32_t nx, ny, nz; } sfw_dims;

typedef struct { float w, mx, my, mz, sigma, d; } sfw_atom;

/* Maximum of the grid certificate: value, grid indices (sigma, d) and voxel. */
typedef struct { float eta; int32_t i_sigma, i_d, x, y, z; } sfw_argmax;

typedef struct sfw_workspace sfw_workspace;
typedef struct sfw_net sfw_net; /* the proposal network (see the end of this header) */

/* Solver options (host memory). sfw_default_options fills the defaults. */
typedef struct {
  int32_t mode;                      /* SFW_MODE_BSFW (default) or SFW_MODE_SFW */
  int32_t n_sigma, n_d;              /* candidate grid sizes (<= SFW_MAX_GRID each) */
  float sigma_grid[SFW_MAX_GRID];    /* default linspace(1, 2, 4) */
  float d_grid[SFW_MAX_GRID];        /* default {1.5, 2, 2.5} */
  float sigma_lo, sigma_hi;          /* box of the domain for sigma, default [0.5, 4] */
  float d_lo, d_hi;                  /* box for d, default [1.2, 3]; centres are boxed
                                        to [0, n-1] on each axis */
  float trunc_T;                     /* grid kernels keep g >= exp(-T) cube, default 12 */
  double eta_tol;                    /* continue while eta* > 1 + eta_tol, default 1e-3 */
  double prune_rel;                  /* drop w <= prune_rel * max w, default 1e-6 */
  double merge_tol;                  /* fuse masses closer than this per coordinate, 5e-2 */
  int32_t max_iter;                  /* outer iterations, default 200 */
  int32_t ascent_max_iter;           /* default 200 */
  int32_t slide_max_iter;            /* default 1000 */
  double ascent_gtol, slide_gtol;    /* projected-gradient tolerances, default 1e-9 */
  double ftol;                       /* relative decrease tolerance, default 1e-12 */
  int32_t lbfgs_memory;              /* curvature pairs kept, default 40 */
  int32_t check_finite;              /* reject NaN/Inf in y and H, default 1 */
  int32_t verbose;                   /* print one line per iteration to stderr */
  sfw_net* proposal;                 /* NULL (default): step 1 seeds the local ascent at the
                                        grid maximum of eta. Else a trained proposal network
                                        (on the workspace's stream) seeds it; when the ascent
                                        from that seed ends at eta* <= 1 + eta_tol, the grid
                                        maximum seeds a second ascent, which decides, and
                                        the grid seeds the rest of that solve */
  const sfw_atom* init_atoms;        /* HOST [n_init] or NULL (default, mu = 0): the measure
                                        the solve starts from (algorithms 1 and 2 start at
                                        mu = 0; a measure returned by an earlier solve, e.g.
                                        one stopped by max_iter, resumes it). w >= 0,
                                        sigma > 0, d > 0, all finite, else SFW_EINVAL;
                                        centres, sigma and d are clipped into the box and
                                        zero weights pruned before the first iteration */
  int32_t n_init;                    /* atoms in init_atoms, 0..max_atoms, default 0 */
  double slide_slope_tol;            /* sliding descents: a step whose criterion stays within
                                        slide_slope_tol |C| of the last one (float32 rounding
                                        of C) is taken on its slope (approximate Wolfe test)
                                        when it fails the sufficient-decrease test; default
                                        1e-6, 0 = sufficient decrease only */
  int32_t graphs;                    /* 1: the (C, grad C) evaluations of a solve whose launch
                                        arguments repeat (the sliding descents) replay one
                                        captured HIP graph; 0 (default): every kernel launched
                                        (the same results bit for bit either way) */
  int32_t autotune;                  /* 1 (default): the render's z planes per thread and the
                                        gradient sums' grid size are timed once per volume
                                        shape and power-of-two atom-count bucket on the
                                        workspace, which keeps the choice (every candidate
                                        gives the same results bit for bit); 0 = defaults */
} sfw_options;

/* Per-solve statistics (host memory). */
typedef struct {
  int32_t iterations;        /* outer iterations run */
  int32_t converged;         /* 1 if stopped on eta* <= 1 + eta_tol */
  int32_t n_atoms;           /* atoms in the returned measure */
  int32_t n_eval_cgrad;      /* evaluations of (C, grad C) */
  int32_t n_eval_eta;        /* evaluations of (eta, grad eta) at a point */
  int32_t n_certificates;    /* grid certificates computed */
  int32_t max_support;       /* largest support size reached */
  double criterion;          /* C of the returned measure */
  double last_eta;           /* eta* of the last iteration */
  double seconds_total, seconds_certificate, seconds_ascent, seconds_lasso, seconds_slide;
  int32_t n_proposals;       /* seeds from the proposal network */
  int32_t n_fallbacks;       /* of which the grid maximum had to replace (0 or 1) */
  int32_t n_graph_replays;   /* (C, grad C) evaluations replayed from a captured graph */
  int32_t n_tunings;         /* launch shapes timed by the autotuner during this solve */
  int32_t n_ascent_iterations; /* quasi-Newton iterations of all local ascents (step 1) */
  int32_t n_slide_iterations;  /* quasi-Newton iterations of all sliding descents */
} sfw_stats;

/* ---------------------------------------------------------------- lifecycle */

/* Fill *opts with the defaults listed above. opts: host. */
int sfw_default_options(sfw_options* opts);

/* Create a workspace on the current HIP device for volumes up to vol_max voxels per axis,
 * PSFs up to psf_max taps per axis and up to max_atoms atoms. All scratch (rendered
 * volume, residual, adjoint, reduction partials, lookup tables and the certificate's
 * Fourier-domain arrays for the reserved grid, LASSO columns) is allocated here once; no
 * other call allocates device memory. stream: the stream every call of this
 * workspace enqueues on (0 = the null stream). */
int sfw_workspace_create(sfw_workspace** ws, sfw_dims vol_max, sfw_dims psf_max,
                         int max_atoms, hipStream_t stream);
void sfw_workspace_destroy(sfw_workspace* ws);
/* Re-point the workspace at another stream of the same device. */
int sfw_workspace_set_stream(sfw_workspace* ws, hipStream_t stream);
/* Thread-local message for the last failing call on this thread ("" if none). */
const char* sfw_last_error(void);

/* ---------------------------------------------------------------- operators */

/* Forward model (section 1.1, observation model): phi_mu = H * sum_n w_n g(theta_n),
 * every atom rendered over every voxel with no truncation.
 * atoms: device [n]; phi_mu: device [V] or NULL (result kept in the workspace). */
int sfw_forward(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol,
                const sfw_atom* atoms, int n, float* phi_mu);

/* Criterion and its analytic gradient (section 1.2 criterion; section 2 analytic
 * gradient): r = y - Phi mu, loss = 1/2 sum r^2 + lambda sum w (float64),
 * grad[n] = dC/d(w, mx, my, mz, sigma, d) of every atom.
 * y: device [V]; r_out: device [V] or NULL; loss_out: device double [1] or NULL;
 * grad_out: device [n] or NULL. n may be 0 (then r = y). */
int sfw_residual_grad(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol,
                      const float* y, float lambda, const sfw_atom* atoms, int n,
                      float* r_out, double* loss_out, sfw_atom* grad_out);

/* Volume adjoint Phi^T on a volume (section 1.2, certificate): q = correlation of r with H.
 * r: device [V]; q_out: device [V]. */
int sfw_adjoint(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol,
                const float* r, float* q_out);

/* Vector-Jacobian product of the forward model (section 1.1 observation model; the analytic
 * derivatives of section 2): for a volume g, grad[n] = d<g, Phi mu>/d(w, mx, my, mz, sigma, d)
 * = sum_s (Phi^T g)(s) d(w_n g_n)(s)/dtheta_n, untruncated. It is what reverse-mode
 * differentiation of sfw_forward needs; with g = r it is minus the data-fit part of the
 * gradient of sfw_residual_grad. The workspace's q becomes Phi^T g.
 * g: device [V]; atoms: device [n]; grad_out: device [n] (not NULL when n > 0). */
int sfw_forward_vjp(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol,
                    const float* g, const sfw_atom* atoms, int n, sfw_atom* grad_out);

/* Grid certificate and its maximum (section 1.3 step 1, lookup table of section 2):
 * eta_ij(m) = (1/lambda) sum_{||t||_inf <= R_ij} g(t; 0, sigma_i, d_j) q(m + t),
 * q = Phi^T r, R_ij = ceil(sigma_i (2T)^(1/d_j)), T = trunc_T (<= 0 selects 12),
 * for every voxel centre m. trunc_T is the one argument beyond the paper's statement: the
 * paper leaves the lookup table's extent open; T sets it (kernel values below exp(-T) are
 * dropped; the default 12 drops values below 6e-6 of the peak). ns * nd <= SFW_CERT_MAX_KERNELS
 * and R_ij <= SFW_CERT_MAX_RADIUS (else SFW_EINVAL). best_out: the maximum of eta (not |eta|) over
 * (i, j, z, y, x); ties go to the lowest C-order flat index.
 * r: device [V], or NULL to use the q = Phi^T r left by the last sfw_residual_grad /
 * sfw_certificate on this workspace; sigma_grid, d_grid: HOST float [ns], [nd]
 * (ns, nd <= SFW_MAX_GRID);
 * eta_out: device [ns][nd][nz][ny][nx] or NULL; best_out: device or HOST [1], or NULL
 * (a host best_out makes the call synchronise before returning). */
int sfw_certificate(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol,
                    const float* r, float lambda, const float* sigma_grid, int ns,
                    const float* d_grid, int nd, float trunc_T, float* eta_out,
                    sfw_argmax* best_out);

/* Certificate at points of the domain and its gradient (section 1.3 step 1, local ascent):
 * eta(theta) = (1/lambda) sum_s g(s; theta) q(s) with q = Phi^T r from the last
 * sfw_residual_grad / sfw_adjoint / sfw_certificate call on this workspace (or the
 * q passed here when not NULL), untruncated.
 * thetas: HOST float [n][5] = (mx, my, mz, sigma, d); eta_out: HOST double [n];
 * grad_out: HOST double [n][5] or NULL. Synchronises the stream. */
int sfw_eta_points(sfw_workspace* ws, sfw_dims vol, const float* q, float lambda,
                   const float* thetas, int n, double* eta_out, double* grad_out);

/* Weights-only LASSO (section 1.3 step 3): w = argmin_{w >= 0} 1/2 ||y - sum w_n a_n||^2
 * + lambda sum w_n, a_n = H * g(theta_n) (unit weight). The Gram matrix and A^T y are
 * accumulated in float64 on the GPU; the non-negative quadratic program is solved in
 * float64 on the host by an active-set method. The atoms' w fields are ignored. Columns and
 * Gram entries are cached in the workspace by atom parameters (exact float match) for the
 * same y (pointer and contents) and H: an atom seen in an earlier call reuses its column, as
 * BSFW needs (its atoms do not move between iterations; pruned atoms just drop out).
 * atoms: device [n]; w_out: device double [n], written in stream order. Synchronises the
 * stream to read the atoms and the Gram rows. */
int sfw_lasso_weights(sfw_workspace* ws, const float* H, sfw_dims psf, sfw_dims vol,
                      const float* y, float lambda, const sfw_atom* atoms, int n,
                      double* w_out);

/* The weights step's quadratic program on the device, for many problems in one launch
 * (algorithm 1 step 3 and algorithm 2 step 3: the criterion of section 1.1 restricted to the
 * weights, whose Gram matrix and linear term sfw_lasso_weights builds): for p = 0..count-1,
 * minimise 1/2 w'G_p w - c_p'w subject to w >= 0, in float64, by the active-set method of the
 * host solver (one workgroup per problem, the Cholesky factor of the passive block in LDS).
 * G: device double [count][kmax][kmax], problem p's matrix in the leading k_p x k_p block (row
 * stride kmax), symmetric (both triangles stored and equal) and positive semi-definite;
 * c: device double [count][kmax] (entries past k_p ignored); k: device int [count] with each
 * k_p in [0, kmax], or NULL for k_p = kmax; kmax in [0, SFW_NNQP_MAX_K]; w: device double
 * [count][kmax], written with the minimisers (zeros past k_p); info: device int [count] or
 * NULL, per problem the number of passive-set solves it took, negated if an iteration cap
 * (4 k_p + 20 steps of either loop) ended it. Enqueued on `stream` and returns without a
 * synchronisation. SFW_EINVAL for count < 0, kmax outside its range or a NULL G, c or w
 * (count = 0 or kmax = 0 is a no-op), SFW_EHIP if the launch fails. */
#define SFW_NNQP_MAX_K 128
int sfw_nnqp_batch(const double* G, const double* c, const int* k, int kmax, int count,
                   double* w, int* info, hipStream_t stream);

/* Certificate at points and its gradient, as sfw_eta_points, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace, no allocation and no synchronisation. Its scratch (per-tile
 * partials, sums, a block counter) is one fixed device array of SFW_NOALLOC_SCRATCH_BYTES per
 * GPU, held until the process ends; every call on a GPU shares it, so calls that overlap on
 * one GPU race (order them on one stream).
 * vol: volume size; q: device [V] (= Phi^T r); lambda > 0; thetas: HOST float [n][5] =
 * (mx, my, mz, sigma, d), finite, sigma > 0, d > 0; n in [1, SFW_NOALLOC_MAX_POINTS];
 * eta_out: device double [n]; grad_out: device double [n][5] or NULL; stream: where the
 * kernels are enqueued (results valid once it reaches them). SFW_EINVAL for invalid
 * arguments or when the tiles the points' atoms cover need more partials than the scratch
 * holds (about 43,000 tiles of 16 x 16 x 32 voxels at 1 point, 5,400 at 8 points). */
#define SFW_NOALLOC_SCRATCH_BYTES (1u << 20)
#define SFW_NOALLOC_MAX_POINTS 8
int sfw_eta_points_noalloc(sfw_dims vol, const float* q, float lambda, const float* thetas,
                           int n, double* eta_out, double* grad_out, hipStream_t stream);

/* ---------------------------------------------------------------- profiling */

/* Per-kernel-class device time recorded with HIP events on the workspace stream between
 * sfw_profile_begin and sfw_profile_end. Classes: "prep", "render", "conv_residual",
 * "conv_adjoint", "conv_forward", "grad", "grad_finalize", "cert_conv", "cert_argmax",
 * "lasso_render", "lasso_conv", "lasso_dots", "hash", "eta_grad", "cert_fft" (the
 * certificate's transforms except the inverse z pass), "cert_zinv" (that pass). A class that
 * covers one kernel ("render", "grad", "grad_finalize", "eta_grad" at up to 8 points,
 * "lasso_conv" for box columns, "cert_argmax", "cert_zinv") is timed by that kernel's own start
 * and stop events, so without the dispatch latency; each other timed launch group costs an
 * event pair on the stream (a few microseconds of device idle), so time only the classes of
 * interest when the surrounding throughput matters. */
#define SFW_PROF_KINDS 16
typedef struct { char name[24]; int32_t launches; double ms; } sfw_prof_entry;

/* Start recording the classes named in `classes` (HOST, comma-separated, e.g.
 * "conv_adjoint,cert_fft"; NULL or "" = every class). Creates the event pool on first use;
 * host call, no device sync. SFW_EINVAL for an unknown class name. */
int sfw_profile_begin(sfw_workspace* ws, const char* classes);
/* Stop, synchronise the stream and write one entry per class with launches > 0 into
 * out (HOST [SFW_PROF_KINDS]); *n_out = entries written. */
int sfw_profile_end(sfw_workspace* ws, sfw_prof_entry* out, int* n_out);

/* ---------------------------------------------------------------- solver */

/* SFW (algorithm 1) or BSFW (algorithm 2) from mu = 0: estimate N and the atoms knowing
 * only y, H and lambda (section 1.1, problem statement).
 * y, H: device; opts: HOST or NULL (defaults); atoms_out: HOST [cap]; n_out: HOST;
 * stats: HOST or NULL. Returns SFW_OK, SFW_ENOCONV (cap on iterations, result still
 * written), SFW_ECAP (more than cap atoms; *n_out = needed) or an error. */
int sfw_solve(sfw_workspace* ws, const float* y, sfw_dims vol, const float* H,
              sfw_dims psf, float lambda, const sfw_options* opts, sfw_atom* atoms_out,
              int cap, int* n_out, sfw_stats* stats);

/* One independent problem of a batch: the arguments and outputs of one sfw_solve call.
 * y, H: device; atoms_out: HOST [cap]; n_out: HOST; stats: HOST or NULL; status: written
 * with that solve's return code. */
typedef struct {
  const float* y;
  sfw_dims vol;
  const float* H;
  sfw_dims psf;
  float lambda;
  sfw_atom* atoms_out;
  int32_t cap;
  int32_t* n_out;
  sfw_stats* stats;
  int32_t status;
} sfw_batch_item;

/* Solves n independent problems (many small volumes, each too small to fill the GPU on its
 * own) on n_ws workspaces: one host thread per workspace takes the next unsolved item and
 * runs sfw_solve on it, each workspace on its own stream, so the solves overlap on the GPU.
 * Every workspace must fit every item (vol_max, psf_max, max_atoms); the results of an item
 * do not depend on which workspace solved it. ws: HOST [n_ws]; items: HOST [n]; opts: HOST or
 * NULL (shared by all items). Returns SFW_OK when every item returned SFW_OK, else the code of
 * the first item (in item order) that did not, with sfw_last_error naming it; every item's
 * status is written either way. Synchronous. */
int sfw_solve_batch(sfw_workspace* const* ws, int n_ws, sfw_batch_item* items, int n,
                    const sfw_options* opts);

/* ---------------------------------------------------------------- proposal network
 *
 * A learned proposal for step 1 of Algorithms 1 and 2 (which take the maximum of the grid
 * certificate): four 3x3x3 convolutions with 32 channels, the first of stride 2, ReLU between,
 * reading x = scale * Phi^T r (scale = 1 / lambda gives the certificate's units) and producing
 * on the half-resolution grid ((n + 1) / 2 per axis; voxel o at full-resolution position 2 o)
 * a centre heatmap logit and sigma and d maps. bf16 weights and activations, float32
 * accumulation, on the matrix cores; trained by sfw_net_train_step on these kernels.
 * Parameters (HOST float32, sfw_net_num_params() values): per layer the weights
 * [co][ci][tz][ty][tx] then the biases [co], layers (co, ci) = (32, 1), (32, 32), (32, 32),
 * (3, 32). The solver uses a network through sfw_options.proposal. */
int sfw_net_num_params(void);
/* Network buffers for volumes up to vol_max voxels, on the current device; every call
 * enqueues on `stream` (0 = the null stream). Parameters start at zero. */
int sfw_net_create(sfw_net** net, sfw_dims vol_max, hipStream_t stream);
void sfw_net_destroy(sfw_net* net);
/* Copy the parameters in (and reset the optimizer state) or out; count must equal
 * sfw_net_num_params(). Synchronous. */
int sfw_net_set_params(sfw_net* net, const float* params, int count);
int sfw_net_get_params(sfw_net* net, float* params, int count);
/* out (device f32 [(nz+1)/2][(ny+1)/2][(nx+1)/2][4]): heatmap logit, sigma, d, unused per
 * half-resolution voxel, for the device volume x [nz][ny][nx] times scale. Asynchronous. */
int sfw_net_forward(sfw_net* net, const float* x, sfw_dims vol, float scale, float* out);
/* Loss and gradients against the k (<= 96) atoms still to be found (HOST rows w, mx, my, mz,
 * sigma, d): L = mean over half-resolution voxels of (h - T)^2 + M ((sigma_hat - S)^2 +
 * (d_hat - D)^2), T the maximum of unit Gaussian blobs at the half-resolution centres, M = 1
 * within one voxel of the nearest centre, whose sigma and d are S and D. loss (HOST, nullable),
 * grads (HOST [num_params], nullable). Synchronous. */
int sfw_net_gradients(sfw_net* net, const float* x, sfw_dims vol, float scale, const float* atoms,
                      int k, double* loss, float* grads);
/* One Adam step (beta 0.9, 0.999) of the same loss with learning rate lr; loss (HOST,
 * nullable: the call then returns without synchronising). */
int sfw_net_train_step(sfw_net* net, const float* x, sfw_dims vol, float scale,
                       const float* atoms, int k, float lr, double* loss);
/* The proposal: theta (HOST [5]) = (mx, my, mz, sigma, d) at the heatmap maximum (ties to the
 * lowest voxel); the centre is refined along each axis by the peak of the parabola through
 * log max(h, 1e-3) at the maximum and its two neighbours (at most half a voxel), since the
 * heatmap is fitted to unit Gaussian blobs. score (HOST) = the heatmap there. When no heatmap
 * value is finite (a diverged network) there is no proposal: score = -INFINITY, theta = NaN,
 * and the solver seeds that iteration at the grid maximum instead. Synchronous. */
int sfw_net_propose(sfw_net* net, const float* x, sfw_dims vol, float scale, double* theta,
                    double* score);

#ifdef __cplusplus
}
#endif

#endif /* SFW_H */
