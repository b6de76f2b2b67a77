// Internal declarations of libsfw: workspace layout, per-atom constants, kernel launchers.
// Not part of the public interface (include/sfw.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "sfw.h"

namespace sfw {

// Per-atom constants consumed by the render and reduction kernels. With l = log2(r^2):
//   u * log2(e) = exp2(hd * l + c)        (u = ||s - m||^d / (2 sigma^d))
//   u * log2(e) / r^2 = exp2(hdm1 * l + c)
// where hd = d / 2, hdm1 = hd - 1 and c = -d log2(sigma) - 1 + log2(log2(e)).
// Per-atom constants of the render / gradient kernels: weight, centre, d/2, d/2 - 1,
// c = -d log2(sigma) - 1 + log2(log2 e) (so u log2 e = exp2(d/2 log2 r^2 + c)), and rcut2, the
// squared radius beyond which the atom is exactly zero in float32 (see kAtomCutU).
struct AtomK {
  float w, mx, my, mz, hd, c, hdm1, rcut2;
};

// u = (r / sigma)^d / 2 at which an atom's value exp(-u) = exp2(-u log2 e) is exactly zero in
// float32: 2^-158 is below the smallest denormal, with room for the approximate log2 / exp2.
constexpr double kAtomCutU = 110.0;
// Squared cut radius sigma (2 kAtomCutU)^(1/d), widened by a relative 1e-4 and 1e-3 voxel.
__host__ __device__ inline float atom_rcut2(double sigma, double d) {
  const double r = sigma * pow(2.0 * kAtomCutU, 1.0 / d) * 1.0001 + 1e-3;
  return (float)(r * r);
}

// u beyond which a LASSO column treats its unit atom as zero: exp(-28) < 7e-13 of the peak.
// The dropped tail carries less than about 1e-10 of the atom's mass for every d in the
// domain (the tail of Gamma(3 / d) beyond u), so Gram entries and <a, y> move by far less than
// the float32 rounding of the column itself, while the support box shrinks several-fold.
constexpr double kColumnCutU = 28.0;

// One candidate of the grid-certificate maximum.
struct ArgPart {
  float val;
  int32_t pad;
  long long idx;
};

// Fixed tile shapes of the direct convolution (see launch_conv).
constexpr int kConvTX = 32;
constexpr int kConvTY = 8;
constexpr int kConvRZ = 8;
constexpr int kConvMaxLds = 64 * 1024;
// Largest (16 + px - 1) x (4 + py - 1) input patch of the matrix-core convolution.
constexpr int kMfmaPatchMax = 512;

// Voxel columns of the render kernel: 256 threads over the flattened (y, x) plane,
// kRenderVPT consecutive z per thread by default (4, 8 or 16: the autotuner's candidates).
constexpr int kRenderVPT = 4;
// Gradient-sum kernels: 256 threads over a 16 x 16 tile of (y, x) columns, VPT z per thread.
constexpr int kGradThreads = 256;

// 2^-100: added to the in-plane squared distance so log2(r^2) stays finite at an atom
// centre; every derivative term carrying r^2 then vanishes there as in the limit.
constexpr float kTinyR2 = 7.888609052210118e-31f;

// z stride (floats) of the convolution's staged tile for z-pass size kz (see k_conv).
constexpr int conv_tile_lzp(int kz) {
  int l = (kConvRZ + kz - 1 + 3) / 4 * 4;
  return (l / 4) % 2 == 1 ? l : l + 4;
}

// One axis of a separable FFT: length n = prod(radix), twiddles tw[m] = exp(-2 pi i m / n).
constexpr int kFpParts = 256;  // fingerprint partials per array
constexpr int kAtomArgs = 8;   // atom constants passed by value in one launch
constexpr int kSlotArgs = 128;    // LASSO slot indices passed by value to the Gram-row kernels
constexpr int kDoubleArgs = 128;  // float64 values passed by value to k_store_doubles
struct SlotArgs {
  int s[kSlotArgs];
};
// Completion signal of a kernel whose results the host reads from pinned memory: once every
// block's results are visible at system scope, the last block to finish (counted on ticket, a
// device counter that is 0 between launches) stores seq into *flag (coherent pinned memory),
// so that the host can spin on the flag instead of synchronising the stream. flag == nullptr:
// no signal.
struct SigArgs {
  int* flag;
  unsigned* ticket;
  int seq;
};
constexpr SigArgs kNoSig{nullptr, nullptr, 0};
constexpr int kFftMaxStages = 16;
constexpr int kFftMaxLen = 1024;
constexpr int kFxLines = 16;  // lines (or columns) per block of the fixed-length passes
constexpr int kFftMaxBlur = 256;  // longest transform of the spectral PSF blur
struct FftAxis {
  int n = 1;
  int nstage = 0;
  int radix[kFftMaxStages] = {0};
  int r1 = 0, r2 = 0;  // two-stage fixed-length plan (n = r1 * r2), 0 if none
  const float2* tw = nullptr;
};
struct FftPlan {
  int nx = 0, ny = 0, nz = 0;
  int px = 0;  // x pitch of the spectrum arrays (nx rounded up to 16)
  // The table kernels are real and even in every axis, so are their spectra: one octant
  // (k <= N / 2 on each axis, hx x hy x hz, x fastest) holds each pair spectrum.
  int hx = 0, hy = 0, hz = 0;
  size_t oct = 0;
  FftAxis ax[3];
};

// Spectral PSF blur (see sfw_blur.hip): transform lengths N >= n + (P - 1) / 2 per axis, each
// with a two-stage plan N = r1 r2; half spectrum of hx = N[0] / 2 + 1 columns at a row pitch of
// px elements; spectra laid out [z][N[1]][px].
struct BlurPlan {
  int N[3] = {0, 0, 0};
  int r1[3] = {0, 0, 0}, r2[3] = {0, 0, 0};
  int hx = 0, px = 0;
  bool fused = false;  // x and y of each plane in one block (plane held in LDS)
  bool chain = false;  // residual and the adjoint's forward transform in one plane pass
  size_t lds = 0;      // dynamic LDS bytes of the fused passes
};

struct ConvPlan {
  int px = 1, py = 1, pz = 1;  // kernel taps per axis
  int kz = 4;                  // z taps per LDS pass (template parameter)
  int kzp = 4;                 // pz padded to a multiple of kz
  int kyc = 1;                 // y taps per LDS pass
  size_t lds_bytes = 0;
  dim3 grid;
  int nblocks = 0;
};

enum ProfKind {
  kProfPrep = 0, kProfRender, kProfConvResidual, kProfConvAdjoint, kProfConvForward, kProfGrad,
  kProfGradFinalize, kProfCertConv, kProfCertArgmax, kProfLassoRender, kProfLassoConv,
  kProfLassoDots, kProfHash, kProfEtaGrad, kProfCertFft, kProfCertZinv, kProfCount
};
constexpr int kProfPool = 16384;

// Tiles of the gradient sums at a few points (k_grad_points).
struct GradPlan {
  int vpt = 16;       // z voxels per thread (template parameter)
  int ntile_xy = 0;   // 16 x 16 (y, x) tiles covered
  int ntile_z = 0;
  int ntiles = 0;     // ntile_xy * ntile_z
  // covered region: x tiles [rx0, rx0 + rtx), y tiles from ry0, z tiles from rz0
  int rx0 = 0, ry0 = 0, rtx = 1, rz0 = 0;
};

}  // namespace sfw

struct sfw_workspace {
  int device = 0;
  hipStream_t stream = nullptr;
  sfw_dims vol_max{0, 0, 0};
  sfw_dims psf_max{0, 0, 0};
  int max_atoms = 0;
  size_t vcap = 0;

  // volumes [vcap]
  float* f = nullptr;    // rendered sum of atoms
  float* phi = nullptr;  // H * f
  float* r = nullptr;    // residual y - H * f
  float* q = nullptr;    // Phi^T r
  float* tmpv = nullptr; // LASSO column under construction, misc
  bool q_valid = false;

  // PSF copies in [ky][kx][kzp] layout: forward (convolution) and adjoint (correlation)
  float* wt_fwd = nullptr;
  float* wt_adj = nullptr;
  size_t wt_cap = 0;
  // matrix-core A operands of the same two kernels (used when mfma_conv_ok)
  float* am_fwd = nullptr;
  float* am_adj = nullptr;

  // lookup table of the grid certificate: concatenated [ky][kx][kzp] kernels
  float* lut = nullptr;
  size_t lut_cap = 0;
  std::vector<size_t> lut_off;
  std::vector<int> lut_r;
  std::vector<float> lut_key;  // (T, ns, nd, sigmas..., ds..., volume) of the cached table
  // Fourier-domain certificate: plan, twiddles, spectrum of q, work array and the table
  // spectra paired two per complex array
  sfw::FftPlan fft;
  bool fft_ready = false;
  float2* fft_tw = nullptr;      // [nx + ny + nz]
  float2* fft_qhat = nullptr;    // [N]
  float2* fft_work = nullptr;    // [npairs][N]
  float2* fft_pairs = nullptr;   // [npairs][oct] pair spectra (octants, dense)
  size_t fft_cap = 0;            // complex elements per array (reserved at creation)
  size_t fft_oct_cap = 0;        // complex elements per pair octant (reserved)
  int fft_npairs_cap = 0;

  // spectral PSF blur: spectrum work array [nz][N1][px], PSF spectrum [N2][N1][px] and the
  // twiddles of the three transform lengths in blur_tw_key ([3][kFftMaxBlur])
  float2* blur_spec = nullptr;
  float2* blur_hhat = nullptr;
  float2* blur_tw = nullptr;
  size_t blur_spec_cap = 0, blur_hhat_cap = 0;  // complex elements
  int blur_tw_key[3] = {0, 0, 0};
  float* blur_hcache = nullptr;  // [kHcacheFloats] PSF and grid of the stored spectrum
  int* eta_ticket = nullptr;     // [1] block counter of the one-launch eta evaluation (0 at rest)
  unsigned* sig_ticket = nullptr;  // [1] block counter of the completion signal (0 at rest)
  int* sig_flag = nullptr;         // coherent pinned host word the signalling kernels write
  int sig_seq = 0;                 // sequence number of the last armed signal
  unsigned long long* fp_part = nullptr;  // [2 kFpParts] fingerprint partials (device)
  // [max_atoms][6] (device): the box each LASSO column slot is valid on; the slot holds
  // stale values outside it, which the Gram-row kernels never read
  int* slot_box = nullptr;
  sfw::SigArgs cert_sig = sfw::kNoSig;  // signal of the last certificate maximum (pinned_best)
  sfw::SigArgs sums_sig = sfw::kNoSig;  // signal of the last (C, grad C) sums in host memory
  int* blur_changed = nullptr;   // [1]

  // atoms
  sfw_atom* atoms_dev = nullptr;  // [max_atoms + 1] staging for host-provided atoms
  sfw::AtomK* ak = nullptr;       // [max_atoms + 1]

  // reduction partials
  float* gpart = nullptr;   // gradient partials: [items][6], or [tiles][atoms][6] (points)
  size_t gpart_cap = 0;     // floats
  int* gitem = nullptr;     // [max_atoms + 1] first item of each atom (launch_grad_items)
  double* dpart = nullptr;  // loss / dot partials
  size_t dpart_cap = 0;     // doubles
  double* dres = nullptr;   // [8 * (max_atoms + 2) + 64] float64 results
  sfw::ArgPart* apart = nullptr;
  size_t apart_cap = 0;
  sfw_argmax* best = nullptr;  // [1]

  // LASSO columns a = H * g of unit atoms, cached by atom parameters: slot s of cols
  // [max_atoms][vcap] holds the column of slot_theta[s] when slot_ok[s]; gram_ok[s][t] marks
  // the valid entries of lasso_G (indexed by slot) and lasso_b[s] = <a_s, y>. All of it holds
  // for the y / H fingerprints, shapes and convolution kind below.
  float* cols = nullptr;
  int* lasso_slots = nullptr;  // device [max_atoms]: slot list of the Gram rows being computed
  const float* lasso_y = nullptr;
  unsigned long long lasso_yhash = 0, lasso_hhash = 0;
  sfw_dims lasso_vol{0, 0, 0}, lasso_psf{0, 0, 0};
  bool lasso_mfma = false;
  std::vector<float> slot_theta;         // [max_atoms][5]
  std::vector<char> slot_ok, gram_ok;    // [max_atoms], [max_atoms][max_atoms]
  std::vector<double> lasso_G, lasso_b;  // [max_atoms][max_atoms], [max_atoms]

  // pinned host staging (doubles), carved into regions that never overlap:
  //   [hp_hash, +2) fingerprints of y and H, directly followed by
  //   [hp_atoms, +3 na) atom readback / upload (sfw_atom)
  //   [hp_stage, +4 na) atom constants (AtomK) | [hp_sums, +6 na + 8) reduction sums
  //   [hp_rows, ...) Gram rows | [hp_slots, ...) slot list
  //   [hp_best, +4) certificate maximum
  double* hpin = nullptr;
  size_t hpin_cap = 0;
  size_t hp_hash = 0, hp_atoms = 0, hp_stage = 0, hp_sums = 0, hp_rows = 0;
  size_t hp_slots = 0;  // [max_atoms] int32 slot list on its way to lasso_slots
  size_t hp_best = 0;   // sfw_argmax written by the certificate's final kernel

  // optional per-kernel-class event timing (sfw_profile_begin / end)
  // The solver's (C, grad C) chain (render, blur with residual, adjoint, gradient sums),
  // captured once its launch arguments repeat and replayed while they stay the same (key).
  // Captured on cap_stream (work recorded there is never run there); replayed on `stream`.
  bool graphs = false;  // set by sfw_solve for its duration (sfw_options.graphs)

  // Autotuned launch shapes of the (C, grad C) chain per (volume shape, atom-count bucket):
  // the render's z planes per thread and the gradient sums' grid size, chosen by timing every
  // candidate once on the workspace's own buffers (ws->tune_on, set by sfw_solve from
  // sfw_options.autotune). Every candidate gives the same results bit for bit.
  struct TuneChoice {
    int render_vpt = sfw::kRenderVPT;
    int grad_blocks = 2048;
  };
  std::map<std::vector<int>, TuneChoice> tune;
  bool tune_on = false;
  int tune_runs = 0;
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t cg_exec = nullptr;
  std::vector<long long> cg_key, cg_seen;
  int cg_replays = 0, cg_captures = 0;

  bool prof_on = false;
  unsigned prof_mask = 0;  // bit k: class k is timed
  int prof_used = 0;
  bool prof_overflow = false;
  std::vector<hipEvent_t> prof_start, prof_stop;
  std::vector<int> prof_kind;
};

// the stream a proposal network enqueues on (sfw_cnn.hip)
hipStream_t net_stream(const sfw_net* n);

// the certificate maximum as the final kernel left it in pinned host memory (valid once the
// stream has been synchronised)
inline sfw_argmax* pinned_best(sfw_workspace* ws) {
  return reinterpret_cast<sfw_argmax*>(ws->hpin + ws->hp_best);
}

namespace sfw {
// Records a start event on construction and a stop event on destruction when profiling is on.
// Optional start and stop events of one kernel launch: a profiling class that covers a single
// kernel hands them to the launch, which has them stamped with the kernel's own start and end
// (hipExtLaunchKernelGGL, from <hip/hip_ext.h>, which the HIP sources that expand SFW_LAUNCH
// include); without them the launch is an ordinary one (graph capture included).
struct KernelEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};
#define SFW_LAUNCH(ev, kernel, grid, block, lds, st, ...)                                   \
  do {                                                                                       \
    if ((ev).start || (ev).stop)                                                             \
      hipExtLaunchKernelGGL(kernel, grid, block, lds, st, (ev).start, (ev).stop, 0,          \
                            __VA_ARGS__);                                                    \
    else                                                                                     \
      hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__);                         \
  } while (0)
// For a launcher that has nothing to launch: records the events, so that they stay valid.
inline hipError_t record_events(const KernelEvents& ev, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (ev.start) e = hipEventRecord(ev.start, st);
  if (e == hipSuccess && ev.stop) e = hipEventRecord(ev.stop, st);
  return e;
}

struct ProfScope {
  sfw_workspace* ws;
  int slot = -1;
  bool at_kernel = false;
  // at_kernel: the scope covers one kernel launched with start() and stop() as its own
  // start and stop events (hipExtLaunchKernelGGL), which time the kernel itself, without the
  // dispatch latency that an event pair recorded around the launch also holds; the launch
  // (or its caller) must record both
  ProfScope(sfw_workspace* w, int kind, bool kernel_events = false) : ws(w) {
    if (!ws->prof_on || !((ws->prof_mask >> kind) & 1u)) return;
    if (ws->prof_used >= (int)ws->prof_start.size()) {
      ws->prof_overflow = true;
      return;
    }
    slot = ws->prof_used++;
    ws->prof_kind[slot] = kind;
    at_kernel = kernel_events;
    if (!at_kernel) (void)hipEventRecord(ws->prof_start[slot], ws->stream);
  }
  hipEvent_t start() const { return slot >= 0 && at_kernel ? ws->prof_start[slot] : nullptr; }
  hipEvent_t stop() const { return slot >= 0 && at_kernel ? ws->prof_stop[slot] : nullptr; }
  KernelEvents events() const { return KernelEvents{start(), stop()}; }
  ~ProfScope() {
    if (slot >= 0 && !at_kernel) (void)hipEventRecord(ws->prof_stop[slot], ws->stream);
  }
};
}  // namespace sfw

namespace sfw {

// ---- error plumbing (sfw_api.cpp)
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
// A new completion signal of the workspace (next sequence number) for one launch of a kernel
// that writes results for the host.
SigArgs sig_arm(sfw_workspace* ws);
// Waits until the kernel launched with s has written its results (a host spin on the coherent
// flag; a stream that finishes without the signal is an error); kNoSig: synchronises the
// stream instead.
int sig_wait(sfw_workspace* ws, const SigArgs& s);

#define SFW_HIP(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return sfw::hip_fail(e_, #call); \
  } while (0)

// ---- launchers (sfw_kernels.hip); each returns a hipError_t from the launch
ConvPlan plan_conv(sfw_dims vol, int px, int py, int pz);
// Points-kernel tiles (16 x 16 columns, 32 planes deep, 16 in volumes under 32 planes) that meet box
// {x0, x1, y0, y1, z0, z1} (voxels, half-open).
GradPlan plan_grad_box(sfw_dims vol, const int box[6]);

// One launch: atom constants (atoms may be null when n == 0) and the forward / adjoint PSF
// operands for the matrix-core (mfma) or VALU (kzp) convolution (H may be null).
hipError_t launch_prep(const sfw_atom* atoms, int n, bool unit_weight, AtomK* ak, const float* H,
                       sfw_dims psf, bool mfma, int kzp, bool fwd, bool adj, float* out_fwd,
                       float* out_adj, hipStream_t st);
// dst[0..n) = host[0..n) (at most kAtomArgs atom constants) through kernel arguments.
hipError_t launch_store_atoms(const AtomK* host, int n, AtomK* dst, hipStream_t st);
// dst[0..n) = host[0..n) through kernel arguments (launches of kDoubleArgs values)
hipError_t launch_store_doubles(const double* host, int n, double* dst, hipStream_t st);
// Fingerprints of y and H (partials in part, device [2 kFpParts]) into out[0], out[1], and a
// copy of the n atoms into atoms_out; out and atoms_out may be pinned host memory, signalled
// by sig.
hipError_t launch_fingerprints(const float* y, size_t ny, const float* H, size_t nh,
                               const sfw_atom* atoms, int n, unsigned long long* part,
                               unsigned long long* out, float* atoms_out, const SigArgs& sig,
                               hipStream_t st);
// vpt: z planes per thread, 4, 8 or 16 (the same f bit for bit: every voxel takes its offsets
// to the atom centres from its own coordinates and sums its nonzero atoms in index order,
// whatever the tile).
hipError_t launch_render(const AtomK* ak, int n, sfw_dims vol, float* f, hipStream_t st,
                         int vpt = kRenderVPT, const KernelEvents& ev = {});

enum ConvEpilogue { kEpiPlain = 0, kEpiResidual = 1, kEpiArgmax = 2, kEpiColumn = 3 };
// out = conv(in, W) with W in [ky][kx][kzp] layout (already flipped for a correlation).
//  kEpiPlain:    out[v] = conv (kEpiColumn: the same, for region launches of the matrix-core
//                kernel)
//  kEpiResidual: out[v] = yobs[v] - conv; dpart[block] = sum over the block of out^2
//  kEpiArgmax:   eta = conv * scale; out[v] = eta if out != nullptr;
//                apart[block] = max of eta over the block, flat index idx_base + v
hipError_t launch_conv(const ConvPlan& p, const float* in, const float* wt, sfw_dims vol,
                       int epi, float* out, const float* yobs, double* dpart, float scale,
                       long long idx_base, ArgPart* apart, hipStream_t st);

// Matrix-core convolution for PSFs with pz <= 16 and px * py <= 128 (see k_conv_mfma).
// The A operands (per-lane weights, mfma_steps * 64 floats) are built by launch_prep. kEpiResidual writes one partial per wave: dpart[block * 4 + wave].
bool mfma_conv_ok(int px, int py, int pz);
int mfma_steps(int px, int py);
int mfma_conv_blocks(sfw_dims vol);
hipError_t launch_conv_mfma(const float* in, const float* amat, sfw_dims psf, sfw_dims vol,
                            int epi, float* out, const float* yobs, double* dpart,
                            hipStream_t st);
// Output region of the matrix-core convolution: 16-wide x tiles [tx0, tx1), 4-high y tiles
// [ty0, ty1) and output planes [z0, z1) in chunks of zchunk planes (one per blockIdx.z).
struct ConvRegion {
  int tx0, tx1, ty0, ty1, z0, z1, zchunk;
};
ConvRegion conv_region_full(sfw_dims vol);
// Plain convolution restricted to a region (outputs elsewhere are not written).
hipError_t launch_conv_mfma_region(const float* in, const float* amat, sfw_dims psf, sfw_dims vol,
                                   const ConvRegion& rg, float* out, hipStream_t st);
// out = H * (w g) of the atom *atom on box = [x0, x1, y0, y1, z0, z1) only (H in its [z][y][x]
// layout), the atom computed on the fly; the rest of out is left untouched. column_box_ok: the
// PSF fits the kernel (P_x <= 33, P_z <= 33, LDS tile).
constexpr int kColumnBoxMaxLds = 160 * 1024;
bool column_box_ok(sfw_dims psf);
// box_out (device int[6], may be null) receives the box.
hipError_t launch_column_box(const AtomK* atom, const float* H, sfw_dims psf, sfw_dims vol,
                             const int box[6], float* out, int* box_out, hipStream_t st);
// Up to kBoxColumns such columns (one PSF, each with its atom, box, output and box record) in
// one launch; each column the same as launch_column_box gives it alone.
constexpr int kBoxColumns = 8;
struct ColumnBoxJob {
  const AtomK* atom;
  float* out;
  int* box_out;
  int box[6];
};
hipError_t launch_column_boxes(const ColumnBoxJob* jobs, int n, const float* H, sfw_dims psf,
                               sfw_dims vol, hipStream_t st, const KernelEvents& ev = {});

// The per-atom sums of at most kAtomArgs atoms given by their constants on the host, reduced
// to sums_out[6 a + c] (float64; may be host memory) by the last block; ticket: device int that
// is 0 between launches.
hipError_t launch_grad_points(const GradPlan& p, const AtomK* host_atoms, int n, const float* q,
                              sfw_dims vol, float* gpart, int* ticket, double* sums_out,
                              const SigArgs& sig, hipStream_t st, const KernelEvents& ev = {});
// The gradient sums of the atoms ak[0, n) against q, one partial per item (an atom on one of
// the 16 x 16 x 16 volume tiles its cut ball may reach) at gpart[6 i + c]; atom a's items are
// item_start[a] .. item_start[a + 1] - 1 (device, n + 1 ints, written by the kernel). At most
// n * grad_item_tiles(vol) items. `blocks` (grid size) changes no result.
int grad_item_tiles(sfw_dims vol);
hipError_t launch_grad_items(const AtomK* ak, int n, const float* q, sfw_dims vol, float* gpart,
                             int* item_start, int blocks, hipStream_t st,
                             const KernelEvents& ev = {});
// Sums partials in a fixed order (float64): over the ntiles tiles of the tile layout
// (launch_grad_points), or over the atom's items when item_start is given (launch_grad_items).
// For atom a:
//   sums[a*6 + 0..5] = (S_g, S_u, S_l, S_mx, S_my, S_mz)
// with S_g = sum q g, S_u = sum q g u', S_l = sum q g u' log2 r^2,
// S_m = sum q g u' (s - m) / r^2 and u' = u log2(e). If loss_part != nullptr,
// sums[6 n] = 1/2 sum of the nloss loss partials. If grad_out != nullptr, also writes the
// gradient of C (float) using atoms and lambda, or with vjp the vector-Jacobian product
// sum_s q df/d(w, m, sigma, d) of the forward model (lambda unused).
hipError_t launch_grad_finalize(const float* gpart, int ntiles, const int* item_start, int n,
                                const double* loss_part, int nloss, const sfw_atom* atoms,
                                float lambda, double* sums, sfw_atom* grad_out, double* loss_out,
                                hipStream_t st, bool vjp = false,
                                const SigArgs& sig = kNoSig, const KernelEvents& ev = {});
// The maximum goes to best (device) and, when best_host is not null, to pinned host memory.
hipError_t launch_argmax_final(const ArgPart* apart, int nparts, sfw_dims vol, int nd,
                               sfw_argmax* best, sfw_argmax* best_host, const SigArgs& sig,
                               hipStream_t st, const KernelEvents& ev = {});
// out[c] = sum_v a[v] * cols[c][v] for c < k, out[k] = sum_v a[v] * y[v] (float64).
// dots of column a (valid on abox) with the k columns cols + slot(c) * colstride (each valid
// on its box slot_box[6 slot(c)...], device) and with y (out[k]), a product counting only
// where both factors are valid; slot(c) is sa.s[c] for c < kSlotArgs, else slots[c] (device).
// out may be pinned host memory.
hipError_t launch_dots(const float* a, const int abox[6], const float* cols, const SlotArgs& sa,
                       const int* slots, const int* slot_box, int k, size_t colstride,
                       const float* y, sfw_dims vol, double* dpart, int nblocks, double* out,
                       const SigArgs& sig, hipStream_t st);
// Gram row over box = {x0, x1, y0, y1, z0, z1} (half-open; x0, x1, nx and colstride multiples
// of 4) that holds every nonzero of a.
hipError_t launch_dots_box(const float* a, const float* cols, const SlotArgs& sa,
                           const int* slots, const int* slot_box, int k, size_t colstride,
                           const float* y, sfw_dims vol, const int box[6], double* dpart,
                           int dpart_cap, double* out, const SigArgs& sig, hipStream_t st);
// The Gram rows of up to kDotsRows columns (each with its box, as for launch_dots_box) in one
// launch and one final reduction: row r's sums to out + r out_stride, each row's sums the same
// as launch_dots_box gives it alone.
constexpr int kDotsRows = 8;
struct GramRowBox {
  const float* a;
  int box[6];
};
// blocks (and float64 partials per column) of one row over box
int dots_box_blocks(const int box[6]);
hipError_t launch_dots_box_rows(const GramRowBox* rows, int nr, const float* cols,
                                const SlotArgs& sa, const int* slots, const int* slot_box, int k,
                                size_t colstride, const float* y, sfw_dims vol, double* dpart,
                                int dpart_cap, double* out, size_t out_stride, const SigArgs& sig,
                                hipStream_t st);
// dst[0..6) = box (device)
hipError_t launch_store_box(const int box[6], int* dst, hipStream_t st);
hipError_t launch_any_nonfinite(const float* v, size_t n, int* flag, hipStream_t st);

// ---- Fourier-domain grid certificate (sfw_fft.hip)
bool fft_plan_cert(sfw_dims vol, int rmax, FftPlan& pl);
void fft_twiddles(int n, std::vector<float2>& tw);
hipError_t fft_scatter_pair(const FftPlan& pl, const float* ka, int ra, int kzpa, const float* kb,
                            int rb, int kzpb, float2* out, hipStream_t st);
hipError_t fft_forward_c2c(const FftPlan& pl, float2* data, hipStream_t st);
hipError_t fft_forward_volume(const FftPlan& pl, const float* q, sfw_dims vol, float2* qhat,
                              hipStream_t st);
int fft_argmax_blocks(const FftPlan& pl, sfw_dims vol);
// fixed-length passes (sfw_fft_fixed.hip)
bool fft_fixed_plan(int L, int* r1, int* r2);
// Spectral PSF blur (sfw_blur.hip). blur_plan: false when some axis needs a transform longer
// than kFftMaxBlur or the PSF is deeper than the spectrum kernel supports.
bool blur_plan(const sfw_dims& vol, const sfw_dims& psf, BlurPlan& bp);
hipError_t launch_blur_twiddles(const BlurPlan& bp, float2* tw, hipStream_t st);
// The spectrum is recomputed only when H or the grid differ from the copy in hcache
// ([kHcacheFloats], zeroed at creation); changed: device int scratch.
constexpr int kHcacheFloats = 16 + 32768;
hipError_t launch_psf_spectrum(const BlurPlan& bp, const float* H, sfw_dims psf, float2* hhat,
                               float* hcache, int* changed, hipStream_t st);
// Number of float64 loss partials the residual epilogue writes.
int blur_residual_parts(const BlurPlan& bp, const sfw_dims& vol);
// out = H * in (adjoint = false) or the correlation with H (adjoint = true) on the volume, with
// epilogue kEpiPlain or kEpiResidual (out = yobs - H * in, loss partials into dpart).
// spec: work array; tw: the plan's twiddles; hhat: the PSF spectrum of launch_psf_spectrum.
hipError_t launch_blur(const BlurPlan& bp, const float* in, const sfw_dims& vol,
                       const float2* hhat, bool adjoint, int epi, float* out, const float* yobs,
                       double* dpart, float2* spec, const float2* tw, hipStream_t st);
// When bp.chain: r = yobs - H * f (loss partials into dpart, one per plane) with the forward
// x-y spectrum of r left in spec, then q = Phi^T r from that spectrum.
hipError_t launch_blur_residual_chain(const BlurPlan& bp, const float* f, const sfw_dims& vol,
                                      const float2* hhat, const float* yobs, float* r_out,
                                      double* dpart, float2* spec, const float2* tw,
                                      hipStream_t st);
hipError_t launch_blur_adjoint_chain(const BlurPlan& bp, const sfw_dims& vol, const float2* hhat,
                                     float* q_out, float2* spec, const float2* tw,
                                     hipStream_t st);
hipError_t fx_strided(int L, dim3 grid, hipStream_t st, const float2* src, size_t src_b,
                      float2* dst, size_t dst_b, const float2* tw, int ncols, size_t istride,
                      size_t ostride, int n_in, int n_out);
// ev0, ev1 (optional): the kernel's own start and stop events
hipError_t fx_z_inverse(int L, hipStream_t st, const float2* qhat, const float2* oct,
                        size_t oct_b, int hx, int hy, float2* work, size_t work_b,
                        const float2* tw, int Nx, int Ny, int px, int n_out, int npairs,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t fx_x_real(int L, dim3 grid, hipStream_t st, const float* q, int nx, int ny,
                     const float2* tw, int Ny, int px, float2* out);
hipError_t fx_x_argmax(int L, dim3 grid, hipStream_t st, const float2* work, size_t work_b,
                       int nx, int ny, int nz, const float2* tw, int Ny, int px, float scale,
                       int nslices, float* eta_out, ArgPart* apart, int nblk);
hipError_t fft_pack_octant(const FftPlan& pl, const float2* full, float2* oct, hipStream_t st);
// The inverse side of the certificate in two launch groups: the z pass of every pair
// (fft_inverse_pairs_z) and the y and x passes with the block maxima (fft_inverse_pairs_yx).
// ev0, ev1 (optional): recorded at the start and the end of the z pass (the one kernel's own
// events on the fixed-length path, an event pair around the launch otherwise).
hipError_t fft_inverse_pairs_z(const FftPlan& pl, const float2* qhat, const float2* pairs,
                               float2* work, size_t bstride, int nslices, sfw_dims vol,
                               hipStream_t st, hipEvent_t ev0 = nullptr,
                               hipEvent_t ev1 = nullptr);
hipError_t fft_inverse_pairs_yx(const FftPlan& pl, float2* work, size_t bstride, int nslices,
                                sfw_dims vol, float scale, float* eta_out, ArgPart* apart,
                                int nblk, hipStream_t st);

}  // namespace sfw
