// Batched solves: independent problems on several workspaces at once.
//
// A small volume (tens of thousands of voxels) leaves most of the GPU idle during one solve,
// whose time goes mostly to short kernels separated by host decisions (line searches, the
// weights' NNQP, the grid maximum). Solves of independent volumes share nothing, so one host
// thread per workspace runs sfw_solve on the next unsolved item; each workspace owns its
// stream, pinned staging and completion flag, and the kernels of different solves overlap on
// the device.
#include <hip/hip_runtime.h>

#include <atomic>
#include <string>
#include <thread>
#include <vector>

#include "sfw.h"
#include "sfw_internal.h"

using namespace sfw;

extern "C" int sfw_solve_batch(sfw_workspace* const* ws, int n_ws, sfw_batch_item* items, int n,
                               const sfw_options* opts) {
  try {
    if (n < 0) return fail(SFW_EINVAL, "n must be >= 0");
    if (n == 0) return SFW_OK;
    if (!ws || n_ws < 1) return fail(SFW_EINVAL, "at least one workspace is needed");
    if (!items) return fail(SFW_EINVAL, "items is NULL");
    for (int w = 0; w < n_ws; ++w)
      if (!ws[w]) return fail(SFW_EINVAL, "a workspace pointer is NULL");
    for (int w = 0; w < n_ws; ++w)
      for (int v = w + 1; v < n_ws; ++v)
        if (ws[w] == ws[v]) return fail(SFW_EINVAL, "a workspace appears twice (one thread each)");
    for (int i = 0; i < n; ++i)
      if (!items[i].atoms_out || !items[i].n_out)
        return fail(SFW_EINVAL, "item " + std::to_string(i) + ": atoms_out or n_out is NULL");
    const int threads = n_ws < n ? n_ws : n;
    std::atomic<int> next{0};
    std::vector<std::string> message(n);
    auto worker = [&](int w) {
      // the workspace's device is current for every call this thread makes
      const hipError_t e = hipSetDevice(ws[w]->device);
      for (;;) {
        const int i = next.fetch_add(1);
        if (i >= n) break;
        sfw_batch_item& it = items[i];
        if (e != hipSuccess) {
          it.status = SFW_EHIP;
          message[i] = std::string("hipSetDevice failed: ") + hipGetErrorString(e);
          continue;
        }
        it.status = sfw_solve(ws[w], it.y, it.vol, it.H, it.psf, it.lambda, opts, it.atoms_out,
                              it.cap, it.n_out, it.stats);
        if (it.status != SFW_OK) message[i] = sfw_last_error();
      }
    };
    std::vector<std::thread> pool;
    pool.reserve(threads - 1);
    for (int w = 1; w < threads; ++w) pool.emplace_back(worker, w);
    worker(0);
    for (auto& t : pool) t.join();
    for (int i = 0; i < n; ++i)
      if (items[i].status != SFW_OK)
        return fail(items[i].status, "batch item " + std::to_string(i) + ": " + message[i]);
    return SFW_OK;
  } catch (const std::exception& e) {
    return fail(SFW_EINVAL, std::string("exception in sfw_solve_batch: ") + e.what());
  } catch (...) {
    return fail(SFW_EINVAL, "unexpected exception in sfw_solve_batch");
  }
}
