// sfw_eta_points_noalloc: the certificate at points and its gradient (section 1.3 step 1, the
// local ascent's evaluation) without a workspace and without any allocation, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// Its scratch (per-tile partial sums, the float64 sums, the last-block counter) lives in one
// file-scope device array per GPU, `scratch`, held until the process ends. Host code never
// passes the array's name to a kernel (in host code it is only a stand-in for the symbol):
// each device's address is looked up once with hipGetSymbolAddress, with that device current,
// and kept per device. Calls on one GPU share the array and keep the last call's contents,
// so calls that overlap on one GPU race; order them on one stream.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "sfw.h"
#include "sfw_internal.h"
#include "sfw_ops.h"

namespace sfw {

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

namespace {

// Scratch layout (bytes): [0, 4) last-block counter, [256, 256 + 8 * 6 * kAtomArgs) float64
// sums, [kPartOff, SFW_NOALLOC_SCRATCH_BYTES) float per-tile partials [tile][point][6].
constexpr size_t kSumsOff = 256;
constexpr size_t kPartOff = 1024;
static_assert(kSumsOff + sizeof(double) * 6 * kAtomArgs <= kPartOff, "scratch layout");

static __device__ __align__(256) unsigned char scratch[SFW_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::atomic<unsigned char*> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// This device's address of `scratch` (looked up once per device, with the device current).
int scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(SFW_EINVAL, "device index out of range");
  unsigned char* p = g_scratch[device].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    p = g_scratch[device].load(std::memory_order_relaxed);
    if (!p) {
      void* addr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !addr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
      p = static_cast<unsigned char*>(addr);
      g_scratch[device].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return SFW_OK;
}

__global__ void k_noalloc_clear(int* ticket) {
  if (threadIdx.x == 0) *ticket = 0;
}

struct PointArgs {
  double sigma[kAtomArgs], d[kAtomArgs];
};

// eta = S_g / lambda and grad eta from the float64 sums of each point (the same expressions as
// the workspace path evaluates on the host).
__global__ void k_eta_finish(const double* __restrict__ sums, int n, double lambda, PointArgs pa,
                             double* __restrict__ eta_out, double* __restrict__ grad_out) {
  const int i = threadIdx.x;
  if (i >= n) return;
  const double ln2 = 0.69314718055994531;
  const double* S = sums + 6 * i;
  const double d = pa.d[i], sg = pa.sigma[i];
  eta_out[i] = S[0] / lambda;
  if (grad_out) {
    double* g = grad_out + 5 * i;
    g[0] = d * ln2 * S[3] / lambda;
    g[1] = d * ln2 * S[4] / lambda;
    g[2] = d * ln2 * S[5] / lambda;
    g[3] = (d / sg) * ln2 * S[1] / lambda;
    g[4] = -(0.5 * ln2 * ln2 * S[2] - log(sg) * ln2 * S[1]) / lambda;
  }
}

}  // namespace
}  // namespace sfw

using namespace sfw;

extern "C" int sfw_eta_points_noalloc(sfw_dims vol, const float* q, float lambda,
                                      const float* thetas, int n, double* eta_out,
                                      double* grad_out, hipStream_t stream) {
  try {
    int rc = check_dims(vol, "vol");
    if (rc) return rc;
    rc = check_lambda(lambda);
    if (rc) return rc;
    if (!q || !thetas || !eta_out) return fail(SFW_EINVAL, "q, thetas or eta_out is NULL");
    if (n < 1 || n > SFW_NOALLOC_MAX_POINTS)
      return fail(SFW_EINVAL, "n must be in [1, SFW_NOALLOC_MAX_POINTS]");
    AtomK hk[kAtomArgs];
    PointArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    for (int i = 0; i < n; ++i) {
      const float* t = thetas + 5 * i;
      for (int c = 0; c < 5; ++c)
        if (!std::isfinite(t[c])) return fail(SFW_EINVAL, "thetas hold NaN or Inf");
      if (!(t[3] > 0) || !(t[4] > 0)) return fail(SFW_EINVAL, "sigma and d must be > 0");
      hk[i] = make_atomk(1.0, t[0], t[1], t[2], t[3], t[4]);
      pa.sigma[i] = t[3];
      pa.d[i] = t[4];
    }
    const GradPlan gp = plan_points(hk, n, vol);
    const size_t part_bytes = (size_t)gp.ntiles * n * 6 * sizeof(float);
    if (part_bytes > SFW_NOALLOC_SCRATCH_BYTES - kPartOff)
      return fail(SFW_EINVAL, "the points' tiles need more than the fixed scratch "
                              "(SFW_NOALLOC_SCRATCH_BYTES); use sfw_eta_points");
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    unsigned char* base = nullptr;
    rc = scratch_address(device, &base);
    if (rc) return rc;
    int* ticket = reinterpret_cast<int*>(base);
    double* sums = reinterpret_cast<double*>(base + kSumsOff);
    float* part = reinterpret_cast<float*>(base + kPartOff);
    // the counter must start at zero (the last block of the sums resets it, but the array
    // keeps whatever an earlier call, possibly an interrupted one, left)
    hipLaunchKernelGGL(k_noalloc_clear, dim3(1), dim3(64), 0, stream, ticket);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_noalloc_clear");
    e = launch_grad_points(gp, hk, n, q, vol, part, ticket, sums, kNoSig, stream);
    if (e != hipSuccess) return hip_fail(e, "k_grad_points");
    hipLaunchKernelGGL(k_eta_finish, dim3(1), dim3(64), 0, stream, sums, n, (double)lambda, pa,
                       eta_out, grad_out);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_eta_finish");
    return SFW_OK;
  } catch (...) {
    return fail(SFW_EINVAL, "unexpected exception in sfw_eta_points_noalloc");
  }
}
