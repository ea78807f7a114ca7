// State-vector comparator for the dense regime: <C> of the p=1 QAOA Max-Cut
// state by a full 2^n complex64 state vector. The paper compares its tensor
// network contraction against Hilbert-space simulation and locates the
// crossover in graph degree (Sec. Results); this is the Hilbert-space side,
// written for the GPU, not part of the tensor-network path.
//
//   |psi> = exp(-i beta sum_q X_q) exp(-i gamma sum_E Z_u Z_v) H^n |0>
//   <C>   = sum_x |psi_x|^2 cut(x),  cut(x) = #edges with x_u != x_v
//
// The diagonal layer gives amplitude 2^(-n/2) exp(-i gamma (|E| - 2 cut(x))),
// computed on the fly in the first pass. The mixer is applied K <= 5
// consecutive qubits per pass: each thread holds the 2^K amplitudes that
// differ only in those qubits and applies the K two-level rotations in
// registers (one read and one write of the state per pass; consecutive
// threads touch consecutive addresses above the first group). The last pass
// forms |psi_x|^2 cut(x) in FP64 without storing the state; per-workgroup
// partial sums are added in a fixed order. cut(x) for the 2^K amplitudes of
// a thread: edges inside the rest r of the bits once per thread, edges
// inside the group from a table, edges between the group and r from two
// popcounts per group qubit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace qtn {

constexpr int kSvMaxEdges = 256, kSvMaxK = 5, kSvThreads = 256, kSvMaxQubits = 34;

struct SvPass {
  float2 *a;             // state, 2^n amplitudes
  double *part;          // per-workgroup partial sums of <C> (last pass)
  int n, n_edges, q0;    // qubits, edges, first qubit of the group
  int64_t threads;       // 2^(n - K): amplitude groups of this pass
  int first, last;       // this pass starts from H^n|0> / ends with <C>
  float c, s;            // cos(beta), sin(beta)
  double gamma, amp0;    // gamma, 2^(-n/2)
  uint64_t nr[kSvMaxK];  // per group qubit: its neighbours outside the group
  uint8_t cgg[1 << kSvMaxK];  // per group pattern j: edges inside the group that j cuts
  uint8_t eu[kSvMaxEdges], ev[kSvMaxEdges];  // edges with both ends outside the group
  int n_rr;
};

template <int K>
__global__ __launch_bounds__(kSvThreads) void sv_pass_kernel(SvPass p) {
  constexpr int J = 1 << K;
  __shared__ float2 phase[kSvMaxEdges + 1];
  __shared__ double red[kSvThreads / 64];
  if (p.first) {
    // exp(-i gamma (|E| - 2c)) * 2^(-n/2) for every cut size c
    for (int c = threadIdx.x; c <= p.n_edges; c += kSvThreads) {
      double sn, cs;
      sincos(p.gamma * (double)(p.n_edges - 2 * c), &sn, &cs);
      phase[c] = make_float2((float)(p.amp0 * cs), (float)(-p.amp0 * sn));
    }
    __syncthreads();
  }
  const uint64_t g = (uint64_t)blockIdx.x * kSvThreads + threadIdx.x;
  const bool act = g < (uint64_t)p.threads;  // the last workgroup may be partly idle (small n)
  const uint64_t lo = g & ((1ull << p.q0) - 1ull), hi = g >> p.q0;
  const uint64_t base = lo | (hi << (p.q0 + K));
  // cut sizes of the thread's amplitudes (first and last pass)
  int cut[J];
  if (p.first || p.last) {
    int crr = 0;
    for (int e = 0; e < p.n_rr; ++e) crr += (int)(((base >> p.eu[e]) ^ (base >> p.ev[e])) & 1ull);
    int pc[K][2];
#pragma unroll
    for (int t = 0; t < K; ++t) {
      pc[t][0] = __popcll(p.nr[t] & base);   // group qubit t reads 0: cut edges to rest bits that read 1
      pc[t][1] = __popcll(p.nr[t] & ~base);  // reads 1: cut edges to rest bits that read 0
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      int c = crr + p.cgg[j];
#pragma unroll
      for (int t = 0; t < K; ++t) c += pc[t][(j >> t) & 1];
      cut[j] = c;
    }
  }
  float2 v[J];
#pragma unroll
  for (int j = 0; j < J; ++j)
    v[j] = p.first ? phase[act ? cut[j] : 0] : (act ? p.a[base | ((uint64_t)j << p.q0)] : make_float2(0.f, 0.f));
  // exp(-i beta X) on each group qubit: (v0, v1) -> (c v0 - i s v1, c v1 - i s v0)
#pragma unroll
  for (int t = 0; t < K; ++t)
#pragma unroll
    for (int j = 0; j < J; ++j)
      if (!((j >> t) & 1)) {
        const float2 x0 = v[j], x1 = v[j | (1 << t)];
        v[j] = make_float2(p.c * x0.x + p.s * x1.y, p.c * x0.y - p.s * x1.x);
        v[j | (1 << t)] = make_float2(p.c * x1.x + p.s * x0.y, p.c * x1.y - p.s * x0.x);
      }
  if (!p.last) {
    if (act)
#pragma unroll
      for (int j = 0; j < J; ++j) p.a[base | ((uint64_t)j << p.q0)] = v[j];
    return;
  }
  double acc = 0.0;
  if (act)
#pragma unroll
    for (int j = 0; j < J; ++j) acc += ((double)v[j].x * v[j].x + (double)v[j].y * v[j].y) * cut[j];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kSvThreads / 64; ++w) s += red[w];
    p.part[blockIdx.x] = s;
  }
}

// Sum of the partial sums in index order (one wave, fixed tree).
__global__ __launch_bounds__(64) void sv_sum_kernel(const double *__restrict__ part, int64_t n, double *out) {
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 64) acc += part[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (threadIdx.x == 0) *out = acc;
}

// Passes: groups of consecutive qubits [q0, q0 + K), the first one holding
// the remainder so the last (which writes the partial sums) has K = min(5, n).
static std::vector<std::pair<int, int>> sv_groups(int n) {
  std::vector<std::pair<int, int>> g;
  const int first = n % kSvMaxK ? n % kSvMaxK : std::min(n, kSvMaxK);
  g.emplace_back(0, first);
  for (int q0 = first; q0 < n; q0 += kSvMaxK) g.emplace_back(q0, kSvMaxK);
  return g;
}

static int64_t sv_blocks(int n, int K) {
  return ((int64_t(1) << (n - K)) + kSvThreads - 1) / kSvThreads;
}

int64_t sv_workspace_bytes(int n) {
  if (n < 1 || n > kSvMaxQubits) return -1;
  return (int64_t(8) << n) + 8 * (sv_blocks(n, sv_groups(n).back().second) + 1);
}

int sv_maxcut_p1(int n, const int32_t *edges, int n_edges, double gamma, double beta, void *workspace,
                 int64_t ws_bytes, double *cost, void *stream) {
  if (n < 1 || n > kSvMaxQubits || n_edges < 0 || n_edges > kSvMaxEdges || (n_edges > 0 && !edges) || !workspace ||
      !cost) {
    set_error("tn_sv_maxcut_p1: bad arguments (1..34 qubits, at most 256 edges, non-NULL buffers)");
    return TN_EINVAL;
  }
  if (ws_bytes < sv_workspace_bytes(n)) {
    set_error("tn_sv_maxcut_p1: workspace smaller than tn_sv_workspace_bytes");
    return TN_EINVAL;
  }
  for (int e = 0; e < n_edges; ++e) {
    const int u = edges[2 * e], v = edges[2 * e + 1];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v) {
      set_error("tn_sv_maxcut_p1: edge endpoint out of range or a loop");
      return TN_EINVAL;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  float2 *a = reinterpret_cast<float2 *>(workspace);
  double *part = reinterpret_cast<double *>(reinterpret_cast<char *>(workspace) + (int64_t(8) << n));
  const std::vector<std::pair<int, int>> groups = sv_groups(n);
  int64_t last_blocks = 1;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const int q0 = groups[gi].first, K = groups[gi].second;
    SvPass p{};
    p.a = a;
    p.part = part;
    p.n = n;
    p.n_edges = n_edges;
    p.q0 = q0;
    p.first = gi == 0;
    p.last = gi + 1 == groups.size();
    p.c = (float)std::cos(beta);
    p.s = (float)std::sin(beta);
    p.gamma = gamma;
    p.amp0 = std::sqrt(std::ldexp(1.0, -n));
    auto in_group = [&](int q) { return q >= q0 && q < q0 + K; };
    for (int e = 0; e < n_edges; ++e) {
      const int u = edges[2 * e], v = edges[2 * e + 1];
      const bool gu = in_group(u), gv = in_group(v);
      if (!gu && !gv) {
        p.eu[p.n_rr] = (uint8_t)u;
        p.ev[p.n_rr] = (uint8_t)v;
        ++p.n_rr;
      } else if (gu && !gv) {
        p.nr[u - q0] |= 1ull << v;
      } else if (gv && !gu) {
        p.nr[v - q0] |= 1ull << u;
      } else {
        for (int j = 0; j < (1 << K); ++j) p.cgg[j] += (uint8_t)(((j >> (u - q0)) ^ (j >> (v - q0))) & 1);
      }
    }
    p.threads = int64_t(1) << (n - K);
    const int64_t blocks = sv_blocks(n, K);
    last_blocks = blocks;
    switch (K) {
      case 1: hipLaunchKernelGGL(sv_pass_kernel<1>, dim3((unsigned)blocks), dim3(kSvThreads), 0, st, p); break;
      case 2: hipLaunchKernelGGL(sv_pass_kernel<2>, dim3((unsigned)blocks), dim3(kSvThreads), 0, st, p); break;
      case 3: hipLaunchKernelGGL(sv_pass_kernel<3>, dim3((unsigned)blocks), dim3(kSvThreads), 0, st, p); break;
      case 4: hipLaunchKernelGGL(sv_pass_kernel<4>, dim3((unsigned)blocks), dim3(kSvThreads), 0, st, p); break;
      default: hipLaunchKernelGGL(sv_pass_kernel<5>, dim3((unsigned)blocks), dim3(kSvThreads), 0, st, p); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      set_error(std::string("tn_sv_maxcut_p1: launch: ") + hipGetErrorString(e));
      return TN_EDEVICE;
    }
  }
  hipLaunchKernelGGL(sv_sum_kernel, dim3(1), dim3(64), 0, st, part, last_blocks, cost);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("tn_sv_maxcut_p1: launch: ") + hipGetErrorString(e));
    return TN_EDEVICE;
  }
  return TN_OK;
}

}  // namespace qtn
