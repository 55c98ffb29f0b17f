// kdss_run_static: kdss_run for callers that cannot allocate device memory.
//
// The plan's whole workspace (leaf stream, tables, credits, queue, hot-node
// slots, extraction buffers) lives in one file-scope device array of
// kStaticWorkspaceBytes per GPU, loaded with the library and held until the
// process ends.  Host code never passes the array's name to a kernel or copy:
// on each device the array's device address comes from hipGetSymbolAddress
// (once, with that device current) and only that address is used.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kdss_internal.h"

namespace {

constexpr size_t kStaticWorkspaceBytes = KDSS_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of this device's array (set up on first use).
int static_workspace(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return kdss::fail(KDSS_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return kdss::fail(KDSS_EUNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return kdss::fail(KDSS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return KDSS_OK;
}

}  // namespace

extern "C" {

int kdss_run_static(kdss_plan* p, uint32_t T, const uint64_t* d_r0, void* d_r, uint32_t* d_order,
                    kdss_result* h_res, void* stream) {
  if (!p || !d_r || !d_order || !h_res) return kdss::fail(KDSS_EINVAL, "null argument");
  if (p->ws_bytes > kStaticWorkspaceBytes)
    return kdss::fail(KDSS_ERANGE, "the plan needs " + std::to_string(p->ws_bytes) +
                                       " workspace bytes; the static workspace holds " +
                                       std::to_string(kStaticWorkspaceBytes));
  void* ws = nullptr;
  int rc = static_workspace(&ws);
  if (rc) return rc;
  // the array keeps whatever the last call on this device left: the plan is
  // copied in again and its queue and hot-node slots cleared (kernels, no
  // memset), and the run itself starts from cleared credits and results
  rc = kdss::upload_plan(p, ws, kStaticWorkspaceBytes, stream, true);
  if (rc) return rc;
  // plain launches on the caller's stream only: no graph instantiation, no
  // timing events, no second stream
  const kdss_opts saved = p->opts;
  p->opts.use_graph = 0;
  p->opts.time_kernels = 0;
  p->opts.extract_every = 0;
  p->one_stream = true;
  rc = kdss::run_plan(p, ws, kStaticWorkspaceBytes, T, d_r0, d_r, d_order, h_res, stream);
  p->opts = saved;
  p->one_stream = false;
  return rc;
}

}  // extern "C"
