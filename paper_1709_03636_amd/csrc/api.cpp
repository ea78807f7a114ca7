// C ABI entry points (declared in include/qtn.h). Host-only calls never
// touch the GPU; device calls forward to the batch runtime.
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <string>

#include "internal.hpp"

namespace qtn {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

// runtime.hip
int batch_create(tn_net *const *nets, int n_nets, const double *coef, double offset, int max_sets, tn_batch **out);
int batch_contract(tn_batch *b, const double *params, int n_sets, double *out, double *obj, void *stream);
int batch_grad(tn_batch *b, const double *params, int n_sets, double *out, double *obj, double *grad, double *gnet,
               void *stream);
int batch_grad_noalloc(tn_batch *b, const double *params, int n_sets, double *out, double *obj, double *grad,
                       double *gnet, void *stream);
int batch_run_graph(tn_batch *b, int with_grad, const double *params, int n_sets, double *out, double *obj,
                    double *grad, double *grad_net, void *stream);
int batch_info(const tn_batch *b, tn_batch_stats *s);
int64_t batch_workspace_bytes(const tn_batch *b);
int batch_bind(tn_batch *b, void *ptr, int64_t bytes);
int set_allocator(tn_alloc_fn alloc, tn_free_fn release, void *ctx);
int batch_autotune(tn_batch *b, const double *params, int n_sets, int reps, const char *cache_path, void *stream);
int batch_apply_cache(tn_batch *b, const char *cache_path);
int batch_set_precision(tn_batch *b, int prec);
int batch_kernel_timing(tn_batch *b, int enable);
int batch_kernel_time(tn_batch *b, int kind, int *n, double *total_ms);
void batch_free(tn_batch *b);
int net_contract(Net &net, const double *params, double *out, double *value, double *grad, void *stream);
int net_bind(Net &net, const double *params, int n_sets, void *dst, int64_t *per_set, void *stream);
void net_dev_free(Net &net);
int stream_sync(void *stream);

}  // namespace qtn

using qtn::Net;

struct tn_net : Net {};

#define GUARD(...)                                           \
  try {                                                      \
    __VA_ARGS__                                              \
  } catch (const std::bad_alloc &) {                         \
    qtn::set_error("host out of memory");                    \
    return TN_ENOMEM;                                        \
  } catch (const std::exception &ex) {                       \
    qtn::set_error(std::string("internal error: ") + ex.what()); \
    return TN_EINVAL;                                        \
  }

extern "C" {

const char *tn_last_error(void) { return qtn::g_err.c_str(); }
const char *tn_version(void) { return "qtn-mi355x 0.1 (gfx950)"; }

int tn_build(const tn_gate *gates, int32_t n_gates, int32_t n_qubits, const double *init, const tn_target *target,
             int32_t n_params, int32_t dtype, tn_net **out) {
  GUARD({
    if (!out) {
      qtn::set_error("tn_build: out is NULL");
      return TN_EINVAL;
    }
    std::unique_ptr<tn_net> n(new tn_net());
    int rc = qtn::build_network(gates, n_gates, n_qubits, init, target, n_params, dtype, *n);
    if (rc != TN_OK) return rc;
    *out = n.release();
    return TN_OK;
  })
}

int tn_wires(const tn_net *net, int32_t *n_wires, int32_t *n_tensors, int32_t *endpoints) {
  if (!net) {
    qtn::set_error("tn_wires: NULL network");
    return TN_EINVAL;
  }
  if (n_wires) *n_wires = (int32_t)net->wire_holders.size();
  if (n_tensors) *n_tensors = (int32_t)net->leaves.size();
  if (endpoints)
    for (size_t w = 0; w < net->wire_holders.size(); ++w) {
      const auto &h = net->wire_holders[w];
      endpoints[2 * w] = h.empty() ? -1 : h.front();
      endpoints[2 * w + 1] = h.size() < 2 ? -1 : h.back();
    }
  return TN_OK;
}

int tn_order_stochastic(const tn_net *net, uint64_t seed, int32_t max_rej, int32_t *pi) {
  GUARD({
    if (!net || !pi) {
      qtn::set_error("tn_order_stochastic: NULL argument");
      return TN_EINVAL;
    }
    std::vector<int> p;
    int rc = qtn::order_stochastic(*net, seed, max_rej, p);
    if (rc != TN_OK) return rc;
    std::copy(p.begin(), p.end(), pi);
    return TN_OK;
  })
}

int tn_order_linegraph(const tn_net *net, int32_t trials, double budget_s, uint64_t seed, int32_t *pi) {
  GUARD({
    if (!net || !pi) {
      qtn::set_error("tn_order_linegraph: NULL argument");
      return TN_EINVAL;
    }
    std::vector<int> p;
    int rc = qtn::order_linegraph(*net, trials, budget_s, seed, p);
    if (rc != TN_OK) return rc;
    std::copy(p.begin(), p.end(), pi);
    return TN_OK;
  })
}

int tn_set_order(tn_net *net, const int32_t *pi, int32_t n) {
  GUARD({
    if (!net || (n > 0 && !pi) || n < 0) {
      qtn::set_error("tn_set_order: bad arguments");
      return TN_EINVAL;
    }
    std::vector<int> p(pi, pi + n);
    qtn::Plan fwd, grad;
    int rc = qtn::compile_plan(*net, p, false, fwd);
    if (rc != TN_OK) return rc;
    if (fwd.peak_live_bytes > (double)net->mem_limit) {
      qtn::set_error("tn_set_order: plan needs " + std::to_string((long long)fwd.peak_live_bytes) +
                     " bytes of live intermediates, limit is " + std::to_string((long long)net->mem_limit));
      return TN_ENOMEM;
    }
    rc = qtn::compile_plan(*net, p, true, grad);
    if (rc != TN_OK) return rc;
    qtn::net_dev_free(*net);
    net->order = p;
    net->plan = std::move(fwd);
    net->gplan = std::move(grad);
    net->has_order = true;
    return TN_OK;
  })
}

int tn_set_memory_limit(tn_net *net, uint64_t bytes) {
  if (!net) {
    qtn::set_error("tn_set_memory_limit: NULL network");
    return TN_EINVAL;
  }
  net->mem_limit = bytes;
  return TN_OK;
}

int tn_plan_info(const tn_net *net, tn_plan_stats *out) {
  if (!net || !out) {
    qtn::set_error("tn_plan_info: NULL argument");
    return TN_EINVAL;
  }
  if (!net->has_order) {
    qtn::set_error("tn_plan_info: no order set");
    return TN_EORDER;
  }
  const qtn::Plan &p = net->plan;
  std::memset(out, 0, sizeof(*out));
  out->n_steps = p.n_steps;
  out->n_tensors = (int32_t)net->leaves.size();
  out->n_wires = (int32_t)net->wire_holders.size();
  out->peak_bits = p.peak_bits;
  out->max_rank_wires = p.max_rank_wires;
  out->n_components = p.n_components;
  out->flops = p.flops;
  out->bytes = p.bytes;
  out->peak_live_bytes = p.peak_live_bytes;
  {
    const qtn::Plan &g = net->gplan;
    std::vector<int64_t> off;
    double leaves = 0;
    for (auto &c : net->consts) leaves += (double)c.size();
    for (auto &t : net->ptensors) leaves += std::ldexp(1.0, t.bits);
    out->grad_bytes = (leaves + (double)qtn::layout_buffers(g, (int)g.ops.size(), off)) * net->elem_bytes();
    out->recompute_runs = g.recompute_runs;
  }
  // fused-executor fit: leaves + live intermediates (forward) in 160 KiB
  double leaf = 0;
  for (auto &c : net->consts) leaf += (double)c.size();
  for (auto &t : net->ptensors) leaf += std::ldexp(1.0, t.bits);
  double fwd_bytes = leaf * net->elem_bytes() + p.peak_live_bytes;
  out->lds_bytes = (int32_t)std::min(fwd_bytes, 2e9);
  out->fused = fwd_bytes <= 160.0 * 1024 ? 1 : 0;
  return TN_OK;
}

int tn_plan_steps(const tn_net *net, int32_t *dims) {
  if (!net || !dims) {
    qtn::set_error("tn_plan_steps: NULL argument");
    return TN_EINVAL;
  }
  if (!net->has_order) {
    qtn::set_error("tn_plan_steps: no order set");
    return TN_EORDER;
  }
  for (size_t s = 0; s < net->plan.step_dims.size(); ++s)
    for (int k = 0; k < 3; ++k) dims[3 * s + k] = net->plan.step_dims[s][k];
  return TN_OK;
}

int tn_contract(tn_net *net, const double *params, double *out, void *stream) {
  GUARD({
    if (!net || !out) {
      qtn::set_error("tn_contract: NULL argument");
      return TN_EINVAL;
    }
    return qtn::net_contract(*net, params, out, nullptr, nullptr, stream);
  })
}

int tn_grad(tn_net *net, const double *params, double *value, double *grad, void *stream) {
  GUARD({
    if (!net || !grad) {
      qtn::set_error("tn_grad: NULL argument");
      return TN_EINVAL;
    }
    return qtn::net_contract(*net, params, nullptr, value, grad, stream);
  })
}

int tn_batch_create(tn_net *const *nets, int32_t n_nets, const double *coef, double offset, int32_t max_sets,
                    tn_batch **out) {
  GUARD({ return qtn::batch_create(nets, n_nets, coef, offset, max_sets, out); })
}

int tn_batch_workspace_bytes(const tn_batch *b, int64_t *bytes) {
  if (!b || !bytes) {
    qtn::set_error("tn_batch_workspace_bytes: NULL argument");
    return TN_EINVAL;
  }
  *bytes = qtn::batch_workspace_bytes(b);
  return TN_OK;
}

int tn_batch_set_workspace(tn_batch *b, void *workspace, int64_t bytes) {
  if (!b) {
    qtn::set_error("tn_batch_set_workspace: NULL batch");
    return TN_EINVAL;
  }
  GUARD({ return qtn::batch_bind(b, workspace, bytes); })
}

int tn_set_allocator(tn_alloc_fn alloc, tn_free_fn release, void *ctx) { return qtn::set_allocator(alloc, release, ctx); }

int tn_batch_contract(tn_batch *b, const double *params, int32_t n_sets, double *out, double *obj, void *stream) {
  if (!b) {
    qtn::set_error("tn_batch_contract: NULL batch");
    return TN_EINVAL;
  }
  GUARD({ return qtn::batch_contract(b, params, n_sets, out, obj, stream); })
}

int tn_batch_grad(tn_batch *b, const double *params, int32_t n_sets, double *out, double *obj, double *grad,
                  double *grad_net, void *stream) {
  if (!b) {
    qtn::set_error("tn_batch_grad: NULL batch");
    return TN_EINVAL;
  }
  GUARD({ return qtn::batch_grad(b, params, n_sets, out, obj, grad, grad_net, stream); })
}

int tn_batch_grad_noalloc(tn_batch *b, const double *params, int32_t n_sets, double *out, double *obj, double *grad,
                          double *grad_net, void *stream) {
  if (!b) {
    qtn::set_error("tn_batch_grad_noalloc: NULL batch");
    return TN_EINVAL;
  }
  GUARD({ return qtn::batch_grad_noalloc(b, params, n_sets, out, obj, grad, grad_net, stream); })
}

int tn_batch_run_graph(tn_batch *b, int32_t with_grad, const double *params, int32_t n_sets, double *out, double *obj,
                       double *grad, double *grad_net, void *stream) {
  if (!b) {
    qtn::set_error("tn_batch_run_graph: NULL batch");
    return TN_EINVAL;
  }
  GUARD({ return qtn::batch_run_graph(b, with_grad, params, n_sets, out, obj, grad, grad_net, stream); })
}

int tn_batch_autotune(tn_batch *b, const double *params, int32_t n_sets, int32_t reps, const char *cache_path,
                      void *stream) {
  if (!b) {
    qtn::set_error("tn_batch_autotune: NULL batch");
    return TN_EINVAL;
  }
  GUARD({ return qtn::batch_autotune(b, params, n_sets, reps, cache_path, stream); })
}

int tn_batch_set_precision(tn_batch *b, int32_t mfma_precision) {
  if (!b) {
    qtn::set_error("tn_batch_set_precision: NULL batch");
    return TN_EINVAL;
  }
  return qtn::batch_set_precision(b, mfma_precision);
}

int tn_batch_kernel_timing(tn_batch *b, int32_t enable) {
  if (!b) {
    qtn::set_error("tn_batch_kernel_timing: NULL batch");
    return TN_EINVAL;
  }
  return qtn::batch_kernel_timing(b, enable);
}

int tn_batch_kernel_time(tn_batch *b, int32_t executor, int32_t *n_launches, double *total_ms) {
  if (!b || !n_launches || !total_ms) {
    qtn::set_error("tn_batch_kernel_time: NULL argument");
    return TN_EINVAL;
  }
  int n = 0;
  const int rc = qtn::batch_kernel_time(b, executor, &n, total_ms);
  *n_launches = n;
  return rc;
}

int tn_batch_apply_tuning(tn_batch *b, const char *cache_path) {
  if (!b || !cache_path) {
    qtn::set_error("tn_batch_apply_tuning: NULL argument");
    return TN_EINVAL;
  }
  GUARD({ return qtn::batch_apply_cache(b, cache_path); })
}

int tn_batch_info(const tn_batch *b, tn_batch_stats *out) {
  if (!b || !out) {
    qtn::set_error("tn_batch_info: NULL argument");
    return TN_EINVAL;
  }
  return qtn::batch_info(b, out);
}

int tn_contract_batch(tn_net *const *nets, int32_t n_nets, const double *params, int32_t n_sets, double *out,
                      void *stream) {
  GUARD({
    tn_batch *b = nullptr;
    int rc = qtn::batch_create(nets, n_nets, nullptr, 0.0, n_sets, &b);
    if (rc != TN_OK) return rc;
    rc = qtn::batch_contract(b, params, n_sets, out, nullptr, stream);
    if (rc == TN_OK) {
      // the batch's device arrays must outlive the kernels that read them
      rc = qtn::stream_sync(stream);
    }
    qtn::batch_free(b);
    return rc;
  })
}

int tn_grad_batch(tn_net *const *nets, int32_t n_nets, const double *params, int32_t n_sets, double *out,
                  double *grad_net, void *stream) {
  GUARD({
    tn_batch *b = nullptr;
    int rc = qtn::batch_create(nets, n_nets, nullptr, 0.0, n_sets, &b);
    if (rc != TN_OK) return rc;
    rc = qtn::batch_grad(b, params, n_sets, out, nullptr, nullptr, grad_net, stream);
    if (rc == TN_OK) {
      rc = qtn::stream_sync(stream);
    }
    qtn::batch_free(b);
    return rc;
  })
}

int tn_bind_params(tn_net *net, const double *params, int32_t n_sets, void *dst, int64_t *per_set, void *stream) {
  if (!net) {
    qtn::set_error("tn_bind_params: NULL network");
    return TN_EINVAL;
  }
  GUARD({ return qtn::net_bind(*net, params, n_sets, dst, per_set, stream); })
}

int64_t tn_sv_workspace_bytes(int32_t n_qubits) { return qtn::sv_workspace_bytes(n_qubits); }

int tn_sv_maxcut_p1(int32_t n_qubits, const int32_t *edges, int32_t n_edges, double gamma, double beta,
                    void *workspace, int64_t workspace_bytes, double *cost, void *stream) {
  GUARD({ return qtn::sv_maxcut_p1(n_qubits, edges, n_edges, gamma, beta, workspace, workspace_bytes, cost, stream); })
}

void tn_free(tn_net *net) {
  if (!net) return;
  qtn::net_dev_free(*net);
  delete net;
}

void tn_batch_free(tn_batch *b) { qtn::batch_free(b); }

}  // extern "C"
