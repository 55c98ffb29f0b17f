// Stand-ins for the device half of the library in a host-only build (the
// address and undefined-behaviour sanitizer run of the host sources): a plan
// is freed as usual, and every call that would touch a device reports
// KDSS_EHIP.  Test infrastructure only.
#include "../../paper_2403_05775_amd/csrc/kdss_internal.h"

extern "C" {

void kdss_plan_free(kdss_plan* p) { delete p; }

void kdss_batch_free(kdss_plan* p) { delete p; }

int kdss_plan_upload(kdss_plan*, void*, size_t, void*) { return kdss::fail(KDSS_EHIP, "no device in this build"); }

int kdss_run(kdss_plan*, void*, size_t, uint32_t, const uint64_t*, void*, uint32_t*, kdss_trace_row*, uint32_t,
             kdss_result*, void*) {
  return kdss::fail(KDSS_EHIP, "no device in this build");
}

}  // extern "C"
