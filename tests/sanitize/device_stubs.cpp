// Host-only build of the contraction library for sanitizer runs on a
// machine without a GPU: the device entry points of the runtime are
// replaced by functions that report "no device"; everything the host does
// (network building, orders, plans, batch planning, precision changes) is
// the library's own code.
#include "../../paper_1709_03636_amd/csrc/batch.hpp"

namespace qtn {

static int no_device() {
  set_error("host-only build: no device");
  return TN_EDEVICE;
}

int batch_contract(tn_batch *, const double *, int, double *, double *, void *) { return no_device(); }
int batch_grad(tn_batch *, const double *, int, double *, double *, double *, double *, void *) { return no_device(); }
int batch_grad_noalloc(tn_batch *, const double *, int, double *, double *, double *, double *, void *) { return no_device(); }
int batch_run_graph(tn_batch *, int, const double *, int, double *, double *, double *, double *, void *) {
  return no_device();
}
int batch_autotune(tn_batch *, const double *, int, int, const char *, void *) { return no_device(); }
int batch_apply_cache(tn_batch *, const char *) { return no_device(); }
int batch_set_precision(tn_batch *b, int prec) { return plan_set_precision(b, prec); }
int batch_kernel_timing(tn_batch *, int) { return no_device(); }
int batch_kernel_time(tn_batch *, int, int *, double *) { return no_device(); }
int batch_bind(tn_batch *, void *, int64_t) { return no_device(); }
void batch_free(tn_batch *b) { delete b; }
int set_allocator(tn_alloc_fn, tn_free_fn, void *) { return no_device(); }
int net_contract(Net &, const double *, double *, double *, double *, void *) { return no_device(); }
int net_bind(Net &, const double *, int, void *, int64_t *, void *) { return no_device(); }
void net_dev_free(Net &) {}
int stream_sync(void *) { return no_device(); }
int64_t sv_workspace_bytes(int) { return -1; }
int sv_maxcut_p1(int, const int32_t *, int, double, double, void *, int64_t, double *, void *) { return no_device(); }

}  // namespace qtn

