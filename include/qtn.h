/*
 * qtn.h - C ABI of the MI355X tensor-network contraction library.
 *
 * The library contracts the closed tensor network of a quantum circuit (the
 * method of "qTorch: The quantum tensor contraction handler", Fried, Sawaya
 * et al.) to one scalar: an output amplitude, an output probability or the
 * expectation value of a Pauli string. Every pairwise contraction of a fixed
 * contraction order runs in hand-written gfx950 HIP kernels.
 *
 * Conventions used throughout:
 *  - Complex numbers are interleaved (re, im) doubles on the host.
 *  - Qubits are numbered 0..n_qubits-1. A two-qubit gate matrix has basis
 *    index 2*x_q0 + x_q1 (q0 is the most significant bit).
 *  - Rotations are R_P(theta) = exp(-i theta P / 2), and
 *    TN_ZZ(theta) = exp(-i theta Z(x)Z / 2). A gate's angle is
 *    theta = coeff * params[param], or theta = coeff when param == -1.
 *  - Every function returns TN_OK (0) or a negative error code and leaves the
 *    object unchanged on error; tn_last_error() then gives a message (per
 *    thread). No C++ exception crosses this boundary.
 *  - Ownership: inputs are copied during the call; a tn_net / tn_batch is
 *    owned by the caller and released with tn_free / tn_batch_free.
 *  - Host-only functions (build, orders, plan, info) never touch the GPU, so
 *    they work on machines without one.
 */
#ifndef QTN_H
#define QTN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tn_net tn_net;
typedef struct tn_batch tn_batch;

/* Error codes. */
enum {
  TN_OK = 0,
  TN_EINVAL = -1,  /* bad argument: qubit out of range, q0 == q1, bad kind, bad param index */
  TN_ENOMEM = -2,  /* plan exceeds the memory limit, or a device allocation failed; checked before any launch */
  TN_EORDER = -3,  /* the contraction order is not a permutation of the wire ids, or none is set */
  TN_EDEVICE = -4, /* a HIP call failed; the object is poisoned afterwards */
  TN_ESTATE = -5   /* object poisoned by an earlier device error, or used in the wrong state */
};

/* Gate kinds. */
enum {
  TN_H = 0, TN_X = 1, TN_Y = 2, TN_Z = 3,
  TN_RX = 4, TN_RY = 5, TN_RZ = 6,
  TN_ZZ = 7,   /* exp(-i theta Z(x)Z / 2), a diagonal 4x4 gate */
  TN_CNOT = 8, /* control q0, target q1 */
  TN_CZ = 9,
  TN_U1 = 10,  /* custom 2x2 matrix (row-major, interleaved re/im) */
  TN_U2 = 11,  /* custom 4x4 matrix (row-major, interleaved re/im) */
  /* Quantum channel rho -> sum_k E_k rho E_k^dagger (e.g. noise, Sec. "A note
   * on noise": Kraus operators as superoperators), given as its folded
   * superoperator S: entry [(2a+b)*4 + (2c+d)] maps rho_cd to rho'_ab, i.e.
   * sum_k E_k[a][c] conj(E_k[b][d]) (16 entries, 32 doubles); for two qubits
   * entry [((2a0+b0)*4 + (2a1+b1))*16 + (2c0+d0)*4 + (2c1+d1)] with qubit q0
   * first (256 entries, 512 doubles). Folded modes only (PROBABILITY,
   * EXPECTATION). A channel that is not trace preserving turns the light
   * cone off for the network (it does not reduce to the identity outside
   * the cone). */
  TN_SUPER1 = 12,
  TN_SUPER2 = 13,
  /* The same channels given by their Kraus operators E_k (Sec. "A note on noise": a
   * channel is a set of Kraus operators), folded into the superoperator above
   * by tn_build: matrix holds n_matrices operators one after another, each
   * 2x2 (TN_KRAUS1, 8 doubles) or 4x4 (TN_KRAUS2, 32 doubles, basis index
   * 2*x_q0 + x_q1), row-major, interleaved re/im. */
  TN_KRAUS1 = 14,
  TN_KRAUS2 = 15
};

typedef struct {
  int32_t kind;
  int32_t q0, q1;        /* q1 = -1 for one-qubit gates */
  int32_t param;         /* index into params[], or -1 for a fixed angle */
  double coeff;          /* theta = coeff * params[param] (or coeff when param == -1) */
  const double *matrix;  /* TN_U1 / TN_U2: 8 or 32 doubles; TN_SUPER1 / TN_SUPER2: 32 or 512 doubles;
                            TN_KRAUS1 / TN_KRAUS2: n_matrices x 8 or 32 doubles; copied */
  int32_t n_matrices;    /* TN_KRAUS1 / TN_KRAUS2: number of Kraus operators (>= 1); ignored otherwise */
} tn_gate;

/* What the network computes (Sec. Preliminaries and Sec. "Estimating the
 * answer string" of the paper: the closed network contracts to one scalar). */
enum {
  TN_AMPLITUDE = 0,    /* <x| C |psi0>: single-layer network with dimension-2 wires */
  TN_PROBABILITY = 1,  /* Tr(Pi rho_out), Pi = (x)_q Pi_q; bits[q] = 0 or 1 projects, 2 traces */
  TN_EXPECTATION = 2   /* Tr(P rho_out) for the Pauli string pauli[] (0=I 1=X 2=Y 3=Z) */
};

typedef struct {
  int32_t mode;
  const uint8_t *bits;   /* AMPLITUDE / PROBABILITY: one entry per qubit */
  const uint8_t *pauli;  /* EXPECTATION: one entry per qubit */
  int32_t lightcone;     /* PROBABILITY / EXPECTATION: 1 = drop gates outside the backward
                            light cone of the measured qubits (exact for unitary gates) */
  int32_t diagonal;      /* 1 = gates diagonal in the computational basis (Z, RZ, ZZ, CZ,
                            diagonal custom gates) keep their wires and become tensors of
                            their diagonal on them (4 or 16 entries folded; 2 or 4 unfolded):
                            those wires are hyperedges, and a contraction keeps (does not sum)
                            a shared index that another live tensor still holds. Exact; the
                            paper keeps every gate dense (sparsity is its future work).
                            0 = dense gates, the paper's network. */
} tn_target;

enum { TN_C64 = 0, TN_C128 = 1 };

/* Matrix-core precision of large contractions (complex GEMM steps). complex64:
 * FP32 products (4 real MFMA products per complex product, default) or
 * split-BF16 products (x = hi + lo in bfloat16, hi*hi + hi*lo + lo*hi),
 * both with FP32 accumulation. complex128: FP64 products (4 real MFMA
 * products per complex product) with FP64 accumulation, always. */
enum { TN_MFMA_FP32 = 1, TN_MFMA_BF16X3 = 2, TN_MFMA_FP64 = 3 };

/* Build the closed network of a circuit (Sec. Preliminaries: one node per
 * initial state, gate and measurement; gates in superoperator form, wires of
 * dimension 4, in PROBABILITY/EXPECTATION mode; gate matrices and
 * dimension-2 wires in AMPLITUDE mode).
 *  gates/n_gates: circuit in time order.  init: n_qubits x 2 complex
 *  (interleaved, 4 doubles per qubit) initial product state, or NULL for |0>.
 *  n_params: length of the params vector later passed to the contract calls.
 *  dtype: TN_C64 (complex64 contraction, FP64 final scalars) or TN_C128.
 *  *out receives a new network without an order. */
int tn_build(const tn_gate *gates, int32_t n_gates, int32_t n_qubits, const double *init,
             const tn_target *target, int32_t n_params, int32_t dtype, tn_net **out);

/* Network shape: number of wires and tensors; wire w joins tensors
 * endpoints[2w] and endpoints[2w+1] (endpoints may be NULL). A hyperedge
 * (diagonal mode) reports its first and last holder. */
int tn_wires(const tn_net *net, int32_t *n_wires, int32_t *n_tensors, int32_t *endpoints);

/* Stochastic order (Algorithm 2 of the paper): pick a random remaining wire,
 * accept it if rank(C) - max(rank(A), rank(B)) <= threshold (ranks in
 * wires), else count a rejection; after more than max_rej rejections raise
 * the threshold by one; reset threshold to -1 after each acceptance.
 * max_rej <= 0 means "number of remaining wires". SplitMix64 seeded by seed.
 * pi receives n_wires wire ids (wires contracted together with the chosen
 * one follow it). Host only. */
int tn_order_stochastic(const tn_net *net, uint64_t seed, int32_t max_rej, int32_t *pi);

/* Line-graph order (Algorithm 1 of the paper): build the line graph L(G) of
 * the network (wires are vertices, adjacent when they share a tensor) and
 * eliminate its vertices greedily by minimum fill-in with random
 * tie-breaks; keep the best of `trials` restarts (or restarts until
 * budget_s seconds when trials <= 0) by (peak tensor size, flops). Host only. */
int tn_order_linegraph(const tn_net *net, int32_t trials, double budget_s, uint64_t seed, int32_t *pi);

/* Fix the contraction order: pi must be a permutation of 0..n_wires-1
 * (TN_EORDER otherwise). Wire pi[i] merges its two end tensors, contracting
 * every wire they share (eq. (1)); a wire whose ends were already merged is
 * skipped; scalars of disconnected pieces are multiplied at the end.
 * Compiles the plan; TN_ENOMEM if its peak exceeds the memory limit. */
int tn_set_order(tn_net *net, const int32_t *pi, int32_t n);

/* Device-memory limit for one network and one angle set (default 64 GiB),
 * applied by the next tn_set_order: an order whose forward intermediates
 * exceed it is refused (TN_ENOMEM); when the gradient program, which keeps
 * every forward intermediate for the adjoint steps, would exceed it, the
 * forward steps are cut into runs whose intermediates are recomputed just
 * before their adjoint steps (not in the paper; tn_plan_stats.recompute_runs
 * and grad_bytes report the result). */
int tn_set_memory_limit(tn_net *net, uint64_t bytes);

typedef struct {
  int32_t n_steps;          /* pairwise contractions */
  int32_t n_tensors;        /* leaf tensors */
  int32_t n_wires;
  int32_t peak_bits;        /* largest intermediate: log2(entries) */
  int32_t max_rank_wires;   /* largest intermediate rank counted in wires */
  int32_t n_components;     /* disconnected pieces (scalars multiplied at the end) */
  int32_t fused;            /* 1: the whole network runs inside one workgroup (LDS resident) */
  int32_t lds_bytes;        /* fused executor: LDS bytes per workgroup (forward) */
  double flops;             /* algorithmic: 8 * 2^(|F_A|+|S|+|F_B|) per step, one angle set */
  double bytes;             /* algorithmic: e*(|A|+|B|+|C|) per step, one angle set */
  double peak_live_bytes;   /* largest sum of live intermediates, one angle set */
  double grad_bytes;        /* gradient program: leaves plus the most intermediates and adjoints held at once */
  int32_t recompute_runs;   /* gradient program: forward runs recomputed before their adjoints (1: none) */
  int32_t reserved;
} tn_plan_stats;

int tn_plan_info(const tn_net *net, tn_plan_stats *out);

/* Per-step shapes: for step s, dims[3s..3s+2] = (|F_A|, |S|, |F_B|) in bits. */
int tn_plan_steps(const tn_net *net, int32_t *dims);

/* Contract one network for one parameter vector (host params, n_params
 * doubles) on the given HIP stream (NULL = default); writes the complex
 * scalar to out[0..1] (host) and synchronises the stream. The closed network
 * contracts to one scalar (Sec. Preliminaries): the amplitude <x|C|psi0>,
 * the probability Tr(Pi rho), or the expectation <psi|M|psi> of a Pauli
 * string (Sec. "Estimating the answer string"), by the pairwise
 * contractions of eq. (1) in the order fixed by tn_set_order. One network
 * per launch sequence: the plain path. */
int tn_contract(tn_net *net, const double *params, double *out, void *stream);

/* Value and gradient of Re(scalar) with respect to params (host buffers;
 * grad has n_params entries) by reverse-mode (adjoint) contraction. Not in
 * the paper: the adjoint of each pairwise contraction of eq. (1) is again a
 * contraction of that form (the result's adjoint with the other operand),
 * run over the same order in reverse with the forward intermediates kept;
 * the adjoint of a parametric gate tensor is contracted with its angle
 * derivative. */
int tn_grad(tn_net *net, const double *params, double *value, double *grad, void *stream);

/* Batched execution of many networks (each with an order set) over many
 * parameter vectors. Not in the paper (its networks run one at a time, with
 * the nodes of one network split over CPU threads, Sec. "Threading"): every
 * (network, parameter vector) pair is independent, and a batch runs them all
 * in a few launches. All networks must share n_params and dtype.
 * coef[i] weights network i in the combined objective
 *   obj[s] = offset + sum_i coef[i] * Re(scalar_i(params_s))
 * (QAOA Max-Cut: coef = -1/2, offset = |E|/2). coef may be NULL (all 0).
 * max_sets bounds n_sets of later calls. */
int tn_batch_create(tn_net *const *nets, int32_t n_nets, const double *coef, double offset,
                    int32_t max_sets, tn_batch **out);

/* Device workspace of a batch: every device array it uses (program
 * descriptors and tables, bound tensors, executor arenas, level items and
 * task queue, outputs of its own). *bytes receives the size the batch needs.
 * Host only. */
int tn_batch_workspace_bytes(const tn_batch *b, int64_t *bytes);

/* Bind a caller-owned device buffer of at least tn_batch_workspace_bytes
 * bytes as the batch's workspace (e.g. a torch.empty(bytes, uint8) tensor);
 * the program arrays are uploaded (synchronous). The buffer must outlive the
 * batch or the next call of this function, and no other work may write it.
 * A batch run without a bound workspace gets one from the allocator
 * (tn_set_allocator), owned and freed by the batch. TN_EINVAL when the
 * buffer is NULL or too small. */
int tn_batch_set_workspace(tn_batch *b, void *workspace, int64_t bytes);

/* Device allocator for the library's own device memory (workspaces of
 * batches without a bound one, the one-network path, autotuner scratch):
 * alloc(bytes, ctx) returns device memory or NULL, release(ptr, ctx) frees
 * it. Both NULL restores hipMalloc / hipFree. Process-wide. */
typedef void *(*tn_alloc_fn)(uint64_t bytes, void *ctx);
typedef void (*tn_free_fn)(void *ptr, void *ctx);
int tn_set_allocator(tn_alloc_fn alloc, tn_free_fn release, void *ctx);

/* Forward pass over n_sets parameter vectors. Device pointers:
 *   params: n_sets x n_params doubles (may be NULL when n_params = 0);
 *   out:    n_nets x n_sets complex scalars (2 doubles each, network-major), may be NULL;
 *   obj:    n_sets doubles (combined objective), may be NULL.
 * Asynchronous on `stream`; capturable in a HIP graph. */
int tn_batch_contract(tn_batch *b, const double *params, int32_t n_sets, double *out, double *obj,
                      void *stream);

/* Forward plus adjoint gradient (reverse-mode contraction over the same
 * order, forward intermediates kept as checkpoints): as tn_batch_contract, and
 *   grad:     n_sets x n_params doubles, d obj[s] / d params[s], may be NULL;
 *   grad_net: n_nets x n_sets x n_params doubles, d Re(scalar_i) / d params, may be NULL.
 * The gradient sums run in FP64. */
int tn_batch_grad(tn_batch *b, const double *params, int32_t n_sets, double *out, double *obj,
                  double *grad, double *grad_net, void *stream);

/* tn_batch_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the pass runs in a fixed 64 MiB scratch array that the library holds on
 * each device until the process ends, instead of the batch's workspace. It
 * calls no device allocator and creates no stream or event. Arguments and
 * results as in tn_batch_grad; every launch goes on `stream`. TN_EINVAL when
 * tn_batch_workspace_bytes exceeds 64 MiB. Each call copies the batch's
 * program arrays into the scratch (copies ordered on `stream` that read the
 * batch's host memory: free the batch only after the stream is done). All
 * calls on a device share its scratch: calls that overlap on one device
 * (concurrent streams or threads) race, and a call leaves its data there. */
int tn_batch_grad_noalloc(tn_batch *b, const double *params, int32_t n_sets, double *out, double *obj,
                          double *grad, double *grad_net, void *stream);

/* Replay the forward (with_grad = 0) or forward+gradient (1) pass through a
 * HIP graph captured on first use for these exact pointers and n_sets;
 * arguments as in tn_batch_grad (grad and grad_net are ignored when
 * with_grad = 0). */
int tn_batch_run_graph(tn_batch *b, int32_t with_grad, const double *params, int32_t n_sets,
                       double *out, double *obj, double *grad, double *grad_net, void *stream);

typedef struct {
  int32_t n_nets, n_fused, n_level;   /* networks on the LDS fused and the level-synchronous path */
  int32_t n_levels;                   /* steps of the longest level-executor program (adjoint) */
  int32_t lds_bytes_fwd, lds_bytes_grad;
  int32_t n_programs;                 /* distinct fused programs (identical networks share one) */
  int32_t fused_block;                /* workgroup size of the fused executor */
  int32_t rec_only;                   /* bit 0 / 1: the forward / adjoint fused programs have a lane
                                         record for every op (kernel without the descriptor path) */
  int32_t sets_per_wave_fwd;          /* angle sets one 64-lane wave of the fused executor runs at once: */
  int32_t sets_per_wave_grad;         /* forward / adjoint programs (1, 2 or 4) */
  int32_t n_global;                   /* networks on the global-arena fused executor (too large for
                                         LDS, steps small enough for one workgroup) */
  int32_t n_level_groups;             /* groups of level networks that share one arena region, run
                                         one after another */
  int32_t n_level_tasked;             /* of those, groups run by the task executor (one launch; a
                                         workgroup runs a whole program for one parameter vector);
                                         the others run one launch per step, spread over the chip */
  int32_t n_level_chunked;            /* level networks run alone, in chunks of parameter vectors */
  int32_t level_launches_fwd;         /* kernel launches of the level executor per pass with all */
  int32_t level_launches_grad;        /* parameter vectors: forward / forward+adjoint */
  int32_t level_split_fwd;            /* matrix-core products of grouped level steps whose summed */
  int32_t level_split_grad;           /* index is split over workgroups: forward / forward+adjoint */
  double flops_fwd, bytes_fwd;        /* algorithmic, one parameter vector, all networks */
  double flops_grad, bytes_grad;      /* algorithmic, adjoint sweep only */
  double exec_flops[3], exec_bytes[3];/* algorithmic forward + adjoint, one parameter vector, of the networks on
                                         each executor (TN_EXEC_FUSED, TN_EXEC_LEVEL, TN_EXEC_GLOBAL) */
  double level_mfma_flops;            /* of those on the level executor: the ops on the matrix cores with the
                                         current precision and tuning (real flops, 8 per complex multiply-add) */
} tn_batch_stats;

int tn_batch_info(const tn_batch *b, tn_batch_stats *out);

/* Autotuner (project-written; not in the paper). Times, on this batch and
 * these device parameters, (1) each workgroup size of the fused executor and
 * (2) for each shape class of large contractions on the level executor, the
 * matrix-core kernel against the thin kernel, and keeps the fastest.
 * Synchronous. cache_path (may be NULL): decisions are merged into this text
 * file ("key value" lines). Plan-time work: run it before timing. */
int tn_batch_autotune(tn_batch *b, const double *params, int32_t n_sets, int32_t reps, const char *cache_path,
                      void *stream);

/* Matrix-core precision for this batch's large steps: TN_MFMA_FP32 or
 * TN_MFMA_BF16X3 for a complex64 batch, TN_MFMA_FP64 (the only one) for a
 * complex128 batch; TN_EINVAL otherwise. */
int tn_batch_set_precision(tn_batch *b, int32_t mfma_precision);

/* Apply decisions from an autotuner cache file without timing. */
int tn_batch_apply_tuning(tn_batch *b, const char *cache_path);

/* Executors of a batch, for kernel timing. */
enum {
  TN_EXEC_FUSED = 0,  /* the LDS fused executor's launch */
  TN_EXEC_LEVEL = 1,  /* per level group: the task executor's launch, or the group's item launches */
  TN_EXEC_GLOBAL = 2  /* the global-arena fused executor's launch */
};

/* Kernel timing (profiling aid, not in the paper). With enable = 1, every
 * later eager tn_batch_contract / tn_batch_grad records a pair of HIP events
 * around each executor launch, on the stream that launch goes on (at most
 * 4096 pending pairs per executor; graph captures and
 * tn_batch_grad_noalloc record none). tn_batch_kernel_time waits for one
 * executor's events, returns how many launches were timed and their summed
 * duration in milliseconds, and forgets them. enable = 0 stops recording and
 * drops pending pairs. */
int tn_batch_kernel_timing(tn_batch *b, int32_t enable);
int tn_batch_kernel_time(tn_batch *b, int32_t executor, int32_t *n_launches, double *total_ms);

/* One-shot conveniences: create a transient batch, run, free (tn_batch_contract /
 * tn_batch_grad semantics, not in the paper). Device pointers. */
int tn_contract_batch(tn_net *const *nets, int32_t n_nets, const double *params, int32_t n_sets,
                      double *out, void *stream);
int tn_grad_batch(tn_net *const *nets, int32_t n_nets, const double *params, int32_t n_sets,
                  double *out, double *grad_net, void *stream);

/* Fill the parametric superoperator tensors for n_sets parameter vectors
 * (angle binding) into a device buffer: for each set s and each distinct
 * parametric tensor t of the network, its entries in canonical wire order.
 * Returns the number of complex entries per set in *per_set when dst is NULL.
 * Exposed for testing the binding kernel on its own. */
int tn_bind_params(tn_net *net, const double *params, int32_t n_sets, void *dst, int64_t *per_set,
                   void *stream);

/* State-vector comparator (not the tensor-network path): <C> of the p=1 QAOA
 * Max-Cut state, |psi> = exp(-i beta sum_q X_q) exp(-i gamma sum_E Z_u Z_v)
 * H^n |0>, <C> = sum over edges of (1 - <Z_u Z_v>)/2, by a full 2^n complex64
 * state vector on the GPU (FP32 amplitudes, FP64 accumulation). It is the
 * Hilbert-space simulation the paper weighs tensor-network contraction
 * against (Sec. Results, the crossover in graph degree). n_qubits 1..34;
 * edges: host array of 2 * n_edges qubit indices (at most 256 edges, no
 * loops); workspace: caller-owned device buffer of at least
 * tn_sv_workspace_bytes(n_qubits) bytes, overwritten; cost: device pointer to
 * one double. Asynchronous on stream; TN_EINVAL for bad arguments or a small
 * workspace. */
int64_t tn_sv_workspace_bytes(int32_t n_qubits);
int tn_sv_maxcut_p1(int32_t n_qubits, const int32_t *edges, int32_t n_edges, double gamma, double beta,
                    void *workspace, int64_t workspace_bytes, double *cost, void *stream);

void tn_free(tn_net *net);
void tn_batch_free(tn_batch *b);
const char *tn_last_error(void);
const char *tn_version(void);

#ifdef __cplusplus
}
#endif
#endif
