// Transformation graph over the kernels (Sec. 2): vector-in / vector-out
// nodes owning their FP64 outputs, scalar variables, a configuration stage
// that places every output in one caller-allocated workspace, and lazy
// evaluation in which changing a variable taints only the nodes that depend
// on it.  Each node runs its own (unfused) kernel, so any intermediate output
// can be read back (Sec. 4.2).
//
// Every output is mirrored in host memory (Sec. 4.2: data lives on the
// device and the host, and is copied only when the side that reads it is
// stale).  A node computes on the GPU or, by an explicit per-node (or
// graph-wide) target flag, on the CPU with the host functions below (Sec.
// 4.2: one flag switches the target device of a transformation); inputs are
// brought to the node's side first, and every copy is counted.  The CPU
// forms are part of this library and are chosen only by that flag: nothing
// falls back to them on its own.
//
// Oscillation nodes come fused (P_ee of one baseline, the general P(a -> b))
// and decomposed into formula items (Sec. 4.1: sin^2 and sin 2phi of each
// phase, and a node that combines them with the mixing coefficients), so a
// change of a mixing angle recomputes only the combining node.  A fused
// chain node (the chain kernel: chi^2 and its gradient) carries the gradient
// through the graph in FP64 or mixed precision.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gna_internal.h"
#include "gna_math.h"

namespace gna {
namespace {

enum NodeKind {
  kPoints, kFlux, kOscProb, kSum, kProduct, kIntegrate, kSmear, kScale, kChi2,
  kOscItem, kPeeItems, kProbItems, kProb, kChainNode
};
constexpr int kMaxSumInputs = 64;

struct Geometry {
  gna_model model;
  gna_problem problem;  // pointers below point into the vectors
  std::vector<double> edges, L, wL, data;
  int n_bins = 0, ppb = 0;
  size_t plan_bytes = 0, plan_off = 0, R_off = 0;
  size_t plan_mixed_bytes = 0, plan_mixed_off = 0;
  bool need_mixed = false;
  gna_plan* plan = nullptr;        // FP64 one-point chain plan: the configuration tables
  gna_plan* plan_mixed = nullptr;  // mixed-precision plan of a mixed chain node
  std::vector<double> R_host;      // dense R in host memory (fetched once, for CPU nodes)
  bool R_host_valid = false;
};

struct Node {
  NodeKind kind;
  std::vector<int> inputs;   // node ids
  std::vector<int> vars;     // variable ids
  std::vector<double> w;     // sum weights
  int geom = -1;             // geometry (points-derived nodes)
  double L = 0.0;            // oscillation baseline
  int pair = 0, item = 0;    // formula item: phase pair (21, 31, 32) and sin^2 / sin 2phi
  int alpha = 0, beta = 0, anti = 0;  // flavours of a probability node
  int prec = GNA_FP64;       // chain node
  int64_t n = 0;             // output length
  size_t off = 0;            // output offset in the workspace
  size_t aux_off = 0;        // chain node: its 5 parameters in the workspace
  const double* table = nullptr;  // configuration tables: output lives in a plan
  bool dirty = true;
  int target = GNA_TARGET_GPU;
  double* host = nullptr;    // host mirror of the output (pinned, placed at bind)
  bool host_valid = false, dev_valid = false;
  int64_t evals = 0, d2h = 0, h2d = 0;
  int64_t failovers = 0;     // GPU failures this node recovered from on the CPU
};

struct SumArgs {
  const double* x[kMaxSumInputs];
  double w[kMaxSumInputs];
  int n_in;
};

__global__ void sum_kernel(SumArgs a, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = a.w[0] * a.x[0][i];
  for (int k = 1; k < a.n_in; ++k) s = dfma(a.w[k], a.x[k][i], s);
  out[i] = s;
}

__global__ void product_kernel(const double* __restrict__ a, const double* __restrict__ b,
                               int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}

__global__ void scale_kernel(const double* __restrict__ x, double v, int64_t n,
                             double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v * x[i];
}

// Bin j sums its ppb consecutive quadrature points in order.
__global__ void integrate_kernel(const double* __restrict__ x, int nb, int ppb,
                                 double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb) return;
  const double* xj = x + (int64_t)j * ppb;
  double s = 0.0;
  for (int k = 0; k < ppb; ++k) s += xj[k];
  out[j] = s;
}

// out_i = sum_j R_ij x_j, one wavefront per row; lanes take columns j = lane,
// lane + 64, ... and the partial sums are folded in a fixed order.
__global__ void smear_kernel(const double* __restrict__ R, const double* __restrict__ x, int nb,
                             double* __restrict__ out) {
  const int row = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (row >= nb) return;  // whole wavefronts leave together
  const double* Ri = R + (int64_t)row * nb;
  double s = 0.0;
  for (int j = lane; j < nb; j += kWave) s = dfma(Ri[j], x[j], s);
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
  if (lane == 0) out[row] = s;
}

// Baker-Cousins chi^2 = 2 sum_i [nu_i - d_i + d_i ln(d_i / nu_i)] by one
// work-group: lanes take bins i = tid, tid + 1024, ..., then a fixed-order
// reduction through LDS.  A bin with nu <= 0 makes the result NaN.
__global__ void __launch_bounds__(1024) chi2_kernel(const double* __restrict__ nu,
                                                    const double* __restrict__ d, int nb,
                                                    double* __restrict__ out) {
  __shared__ double part[1024];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 1024) {
    const double v = nu[i], di = d[i];
    const double t = dfma(di, log_pos(di > 0.0 ? di / v : 1.0), v - di);
    s += (v > 0.0) ? t : __builtin_nan("");
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 2.0 * part[0];
}

// One formula item of the Sec. 4.1 probability over energies E: sin^2 phi
// (item 0) or sin 2phi (item 1) of phi = dm2 (K L) / E, the phase rounded as
// in the fused kernels (q = (K L) / E correctly rounded, phi = dm2 q).
__global__ void osc_item_kernel(const double* __restrict__ E, int64_t n, double KL, double dm,
                                int item, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const PhaseTerms<double> t = phase_terms<double>(dm * phase_per_ev2(KL, E[i]));
  out[i] = item == 0 ? t.S : t.T;
}

// delta + sum_t c_t s_t + d_t u_t over three (or six) item vectors.
struct CombineArgs {
  const double* s[3];
  const double* u[3];  // NULL when the probability has no sin 2phi items
  double c[3], d[3];
  double delta;
};

__global__ void combine_kernel(CombineArgs a, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double p = a.delta;
  for (int t = 0; t < 3; ++t) {
    p = dfma(a.c[t], a.s[t][i], p);
    if (a.u[t]) p = dfma(a.d[t], a.u[t][i], p);
  }
  out[i] = p;
}

// Parameters of a chain node, written by a kernel (no host buffer to keep alive).
__global__ void params_kernel(double* __restrict__ out, double a, double b, double c, double d,
                              double e) {
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
    out[2] = c;
    out[3] = d;
    out[4] = e;
  }
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

bool has_cpu_form(NodeKind k) { return k != kPoints && k != kFlux && k != kChainNode; }

// ---- CPU forms (FP64, libm) -------------------------------------------------
// The same definitions as the kernels above and the fused entry points; the
// phase is rounded the same way (one IEEE division, one product).
double host_phase(double KL, double E, double dm) { return dm * (KL / E); }

void cpu_oscprob(const double* E, int64_t n, double L, const double th[4], double* out) {
  double K0, A, B1, B2;
  pee_coefficients(th[2], th[3], &K0, &A, &B1, &B2);
  const double KL = kPhase * L, dm32 = th[1] - th[0];
  for (int64_t i = 0; i < n; ++i) {
    const double q = KL / E[i];
    const double c21 = std::cos(th[0] * q), c31 = std::cos(th[1] * q), c32 = std::cos(dm32 * q);
    out[i] = K0 + A * (c21 * c21) + B1 * (c31 * c31) + B2 * (c32 * c32);
  }
}

void cpu_osc_item(const double* E, int64_t n, double L, double dm, int item, double* out) {
  const double KL = kPhase * L;
  for (int64_t i = 0; i < n; ++i) {
    const double phi = host_phase(KL, E[i], dm);
    const double s = std::sin(phi);
    out[i] = item == 0 ? s * s : std::sin(2.0 * phi);
  }
}

void cpu_prob(const double* E, int64_t n, double L, const double dm[3], double delta,
              const double re[3], const double im[3], double* out) {
  const double KL = kPhase * L;
  for (int64_t i = 0; i < n; ++i) {
    double p = delta;
    for (int t = 0; t < 3; ++t) {
      const double phi = host_phase(KL, E[i], dm[t]);
      const double s = std::sin(phi);
      p += re[t] * (s * s) + im[t] * std::sin(2.0 * phi);
    }
    out[i] = p;
  }
}

double cpu_chi2(const double* nu, const double* d, int nb) {
  double s = 0.0;
  bool bad = false;
  for (int i = 0; i < nb; ++i) {
    if (!(nu[i] > 0.0)) bad = true;
    double t = nu[i] - d[i];
    if (d[i] > 0.0) t += d[i] * std::log(d[i] / nu[i]);
    s += t;
  }
  return bad ? std::nan("") : 2.0 * s;
}

}  // namespace
}  // namespace gna

struct gna_graph {
  std::vector<gna::Node> nodes;
  std::vector<gna::Geometry> geoms;
  std::vector<double> var_value;
  std::vector<std::string> var_name;
  std::vector<std::vector<int>> var_users;  // nodes reading each variable
  std::vector<std::vector<int>> consumers;  // nodes reading each node
  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;
  double* pinned = nullptr;  // every node's host mirror, in page-locked host memory
  bool bound = false;
  bool failover = false;  // recompute a node on the CPU when its GPU form fails
};

namespace gna {
namespace {

int check_node(const gna_graph* g, int id, const char* what) {
  if (id < 0 || id >= (int)g->nodes.size())
    return fail(GNA_E_INVAL, "%s: node %d does not exist", what, id);
  return GNA_OK;
}

int check_var(const gna_graph* g, int id, const char* what) {
  if (id < 0 || id >= (int)g->var_value.size())
    return fail(GNA_E_INVAL, "%s: variable %d does not exist", what, id);
  return GNA_OK;
}

int add_node(gna_graph* g, Node nd, int32_t* out) {
  const int id = (int)g->nodes.size();
  for (int in : nd.inputs) g->consumers[in].push_back(id);
  for (int v : nd.vars) g->var_users[v].push_back(id);
  g->nodes.push_back(std::move(nd));
  g->consumers.emplace_back();
  if (out) *out = id;
  return GNA_OK;
}

int creation_open(const gna_graph* g, int32_t* out, const char* what) {
  if (!g) return fail(GNA_E_INVAL, "%s: graph is NULL", what);
  if (g->bound) return fail(GNA_E_INVAL, "%s: the graph is already bound", what);
  if (!out) return fail(GNA_E_INVAL, "%s: NULL output id", what);
  return GNA_OK;
}

void taint(gna_graph* g, int id) {
  std::vector<int> stack{id};
  while (!stack.empty()) {
    const int k = stack.back();
    stack.pop_back();
    if (g->nodes[k].dirty) continue;  // its consumers are tainted already
    g->nodes[k].dirty = true;
    for (int c : g->consumers[k]) stack.push_back(c);
  }
}

double* dev_ptr(const gna_graph* g, const Node& nd) {
  return nd.table ? const_cast<double*>(nd.table) : (double*)(g->ws + nd.off);
}

// The host mirror of node id, copied from the device if it is stale there.
int ensure_host(gna_graph* g, int id, hipStream_t s) {
  Node& nd = g->nodes[id];
  if (nd.host_valid) return GNA_OK;
  if (!nd.dev_valid) return fail(GNA_E_INVAL, "graph node %d has no valid copy", id);
  int rc = check_hip(hipMemcpyAsync(nd.host, dev_ptr(g, nd), (size_t)nd.n * 8,
                                    hipMemcpyDeviceToHost, s),
                     "hipMemcpyAsync (graph node to host)");
  if (rc || (rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize (graph node to host)")))
    return rc;
  nd.host_valid = true;
  ++nd.d2h;
  return GNA_OK;
}

// The device copy of node id, uploaded from the host mirror if it is stale.
// Synchronous, so the host mirror may change right after.
int ensure_dev(gna_graph* g, int id, hipStream_t s) {
  Node& nd = g->nodes[id];
  if (nd.dev_valid) return GNA_OK;
  if (!nd.host_valid) return fail(GNA_E_INVAL, "graph node %d has no valid copy", id);
  int rc = check_hip(hipMemcpyAsync(dev_ptr(g, nd), nd.host, (size_t)nd.n * 8,
                                    hipMemcpyHostToDevice, s),
                     "hipMemcpyAsync (graph node to device)");
  if (rc || (rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize (graph node to device)")))
    return rc;
  nd.dev_valid = true;
  ++nd.h2d;
  return GNA_OK;
}

// Dense R of a geometry in host memory (one copy, counted on none of the
// nodes: it is a configuration table of the geometry).
int ensure_R_host(gna_graph* g, Geometry& ge, hipStream_t s) {
  if (ge.R_host_valid) return GNA_OK;
  ge.R_host.resize((size_t)ge.n_bins * ge.n_bins);
  int rc = check_hip(hipMemcpyAsync(ge.R_host.data(), g->ws + ge.R_off, ge.R_host.size() * 8,
                                    hipMemcpyDeviceToHost, s),
                     "hipMemcpyAsync (smearing matrix to host)");
  if (rc || (rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize (smearing matrix)")))
    return rc;
  ge.R_host_valid = true;
  return GNA_OK;
}

int compute(gna_graph* g, int id, hipStream_t s);

// Inputs first (each computed at most once), then the node itself.  Node ids
// are topologically ordered (a node's inputs exist before it), so recursion
// depth is bounded by the chain length.
int evaluate(gna_graph* g, int id, hipStream_t s) {
  Node& nd = g->nodes[id];
  if (!nd.dirty) return GNA_OK;
  for (int in : nd.inputs) {
    const int rc = evaluate(g, in, s);
    if (rc) return rc;
  }
  const int rc = compute(g, id, s);
  if (rc) return rc;
  nd.dirty = false;
  ++nd.evals;
  return GNA_OK;
}

double var(const gna_graph* g, const Node& nd, int k) { return g->var_value[nd.vars[k]]; }

int compute_cpu(gna_graph* g, int id, hipStream_t s) {
  Node& nd = g->nodes[id];
  int rc;
  for (int in : nd.inputs)
    if ((rc = ensure_host(g, in, s))) return rc;
  double* out = nd.host;
  auto in_h = [&](int k) { return (const double*)g->nodes[nd.inputs[k]].host; };
  switch (nd.kind) {
    case kOscProb: {
      const double th[4] = {var(g, nd, 0), var(g, nd, 1), var(g, nd, 2), var(g, nd, 3)};
      cpu_oscprob(in_h(0), nd.n, nd.L, th, out);
      break;
    }
    case kSum:
      for (int64_t i = 0; i < nd.n; ++i) {
        double acc = nd.w[0] * in_h(0)[i];
        for (size_t k = 1; k < nd.inputs.size(); ++k) acc = std::fma(nd.w[k], in_h((int)k)[i], acc);
        out[i] = acc;
      }
      break;
    case kProduct:
      for (int64_t i = 0; i < nd.n; ++i) out[i] = in_h(0)[i] * in_h(1)[i];
      break;
    case kScale: {
      const double v = var(g, nd, 0);
      for (int64_t i = 0; i < nd.n; ++i) out[i] = v * in_h(0)[i];
      break;
    }
    case kIntegrate: {
      const Geometry& ge = g->geoms[nd.geom];
      const double* x = in_h(0);
      for (int j = 0; j < ge.n_bins; ++j) {
        double acc = 0.0;
        for (int k = 0; k < ge.ppb; ++k) acc += x[(int64_t)j * ge.ppb + k];
        out[j] = acc;
      }
      break;
    }
    case kSmear: {
      Geometry& ge = g->geoms[nd.geom];
      if ((rc = ensure_R_host(g, ge, s))) return rc;
      const double* x = in_h(0);
      for (int i = 0; i < ge.n_bins; ++i) {
        double acc = 0.0;
        for (int j = 0; j < ge.n_bins; ++j) acc = std::fma(ge.R_host[(size_t)i * ge.n_bins + j], x[j], acc);
        out[i] = acc;
      }
      break;
    }
    case kChi2: {
      const Geometry& ge = g->geoms[nd.geom];
      out[0] = cpu_chi2(in_h(0), ge.data.data(), ge.n_bins);
      break;
    }
    case kOscItem: {
      const double dm21 = var(g, nd, 0), dm31 = var(g, nd, 1);
      const double dm = nd.pair == 0 ? dm21 : (nd.pair == 1 ? dm31 : dm31 - dm21);
      cpu_osc_item(in_h(0), nd.n, nd.L, dm, nd.item, out);
      break;
    }
    case kPeeItems:
    case kProbItems: {
      double delta, c[3], d[3] = {0.0, 0.0, 0.0};
      if (nd.kind == kPeeItems) {
        double K0, A, B1, B2;
        pee_coefficients(var(g, nd, 0), var(g, nd, 1), &K0, &A, &B1, &B2);
        delta = 1.0;
        c[0] = -A;
        c[1] = -B1;
        c[2] = -B2;
      } else {
        const double ang[4] = {var(g, nd, 0), var(g, nd, 1), var(g, nd, 2), var(g, nd, 3)};
        prob_coefficients(nd.alpha, nd.beta, nd.anti, ang, &delta, c, d);
      }
      const bool six = nd.kind == kProbItems;
      for (int64_t i = 0; i < nd.n; ++i) {
        double p = delta;
        for (int t = 0; t < 3; ++t) {
          p = std::fma(c[t], in_h(t)[i], p);
          if (six) p = std::fma(d[t], in_h(3 + t)[i], p);
        }
        out[i] = p;
      }
      break;
    }
    case kProb: {
      const double ang[4] = {var(g, nd, 0), var(g, nd, 1), var(g, nd, 2), var(g, nd, 3)};
      const double dm[3] = {var(g, nd, 4), var(g, nd, 5), var(g, nd, 5) - var(g, nd, 4)};
      double delta, re[3], im[3];
      prob_coefficients(nd.alpha, nd.beta, nd.anti, ang, &delta, re, im);
      cpu_prob(in_h(0), nd.n, nd.L, dm, delta, re, im, out);
      break;
    }
    default:
      return fail(GNA_E_UNSUPPORTED, "graph node %d has no CPU form", id);
  }
  nd.host_valid = true;
  nd.dev_valid = false;
  return GNA_OK;
}

int compute_gpu(gna_graph* g, int id, hipStream_t s) {
  Node& nd = g->nodes[id];
  int rc;
  for (int in : nd.inputs)
    if ((rc = ensure_dev(g, in, s))) return rc;
  double* out = (double*)(g->ws + nd.off);
  auto in_d = [&](int k) { return (const double*)dev_ptr(g, g->nodes[nd.inputs[k]]); };
  const int t = 256;
  switch (nd.kind) {
    case kOscProb: {
      const double th[4] = {var(g, nd, 0), var(g, nd, 1), var(g, nd, 2), var(g, nd, 3)};
      if ((rc = gna_pee(in_d(0), nd.n, 1, &nd.L, nullptr, th, out, GNA_FP64, s))) return rc;
      break;
    }
    case kSum: {
      SumArgs a{};
      a.n_in = (int)nd.inputs.size();
      for (int k = 0; k < a.n_in; ++k) {
        a.x[k] = in_d(k);
        a.w[k] = nd.w[k];
      }
      hipLaunchKernelGGL(sum_kernel, dim3(blocks_for(nd.n, t)), dim3(t), 0, s, a, nd.n, out);
      break;
    }
    case kProduct:
      hipLaunchKernelGGL(product_kernel, dim3(blocks_for(nd.n, t)), dim3(t), 0, s, in_d(0),
                         in_d(1), nd.n, out);
      break;
    case kScale:
      hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(nd.n, t)), dim3(t), 0, s, in_d(0),
                         var(g, nd, 0), nd.n, out);
      break;
    case kIntegrate: {
      const Geometry& ge = g->geoms[nd.geom];
      hipLaunchKernelGGL(integrate_kernel, dim3(blocks_for(ge.n_bins, t)), dim3(t), 0, s, in_d(0),
                         ge.n_bins, ge.ppb, out);
      break;
    }
    case kSmear: {
      const Geometry& ge = g->geoms[nd.geom];
      const int rows_per_group = t / kWave;
      hipLaunchKernelGGL(smear_kernel,
                         dim3((unsigned)((ge.n_bins + rows_per_group - 1) / rows_per_group)),
                         dim3(t), 0, s, (const double*)(g->ws + ge.R_off), in_d(0), ge.n_bins, out);
      break;
    }
    case kChi2: {
      const Geometry& ge = g->geoms[nd.geom];
      const double* d = (const double*)(ge.plan->ws + ge.plan->lay.data);
      hipLaunchKernelGGL(chi2_kernel, dim3(1), dim3(1024), 0, s, in_d(0), d, ge.n_bins, out);
      break;
    }
    case kOscItem: {
      const double dm21 = var(g, nd, 0), dm31 = var(g, nd, 1);
      const double dm = nd.pair == 0 ? dm21 : (nd.pair == 1 ? dm31 : dm31 - dm21);
      hipLaunchKernelGGL(osc_item_kernel, dim3(blocks_for(nd.n, t)), dim3(t), 0, s, in_d(0), nd.n,
                         kPhase * nd.L, dm, nd.item, out);
      break;
    }
    case kPeeItems:
    case kProbItems: {
      CombineArgs a{};
      if (nd.kind == kPeeItems) {
        double K0, A, B1, B2;
        pee_coefficients(var(g, nd, 0), var(g, nd, 1), &K0, &A, &B1, &B2);
        a.delta = 1.0;
        a.c[0] = -A;
        a.c[1] = -B1;
        a.c[2] = -B2;
      } else {
        const double ang[4] = {var(g, nd, 0), var(g, nd, 1), var(g, nd, 2), var(g, nd, 3)};
        prob_coefficients(nd.alpha, nd.beta, nd.anti, ang, &a.delta, a.c, a.d);
      }
      for (int k = 0; k < 3; ++k) {
        a.s[k] = in_d(k);
        a.u[k] = nd.kind == kProbItems ? in_d(3 + k) : nullptr;
      }
      hipLaunchKernelGGL(combine_kernel, dim3(blocks_for(nd.n, t)), dim3(t), 0, s, a, nd.n, out);
      break;
    }
    case kProb: {
      const double ang[4] = {var(g, nd, 0), var(g, nd, 1), var(g, nd, 2), var(g, nd, 3)};
      const double dm[2] = {var(g, nd, 4), var(g, nd, 5)};
      if ((rc = gna_prob(in_d(0), nd.n, nd.alpha, nd.beta, 1, &nd.L, nullptr, ang, dm, nd.anti, out,
                         GNA_FP64, s)))
        return rc;
      break;
    }
    case kChainNode: {
      const Geometry& ge = g->geoms[nd.geom];
      gna_plan* p = nd.prec == GNA_FP64 ? ge.plan : ge.plan_mixed;
      if (!p->shape.mfma) {
        // One point: its parameters go to the kernel by value, no upload.
        const double th[5] = {var(g, nd, 0), var(g, nd, 1), var(g, nd, 2), var(g, nd, 3),
                              var(g, nd, 4)};
        if ((rc = launch_chain(p, nullptr, 1, out, out + 1, nullptr, s, th))) return rc;
      } else {
        double* params = (double*)(g->ws + nd.aux_off);
        hipLaunchKernelGGL(params_kernel, dim3(1), dim3(64), 0, s, params, var(g, nd, 0),
                           var(g, nd, 1), var(g, nd, 2), var(g, nd, 3), var(g, nd, 4));
        if ((rc = check_hip(hipGetLastError(), "graph chain parameters"))) return rc;
        if ((rc = gna_chain_eval(p, params, 1, out, out + 1, nullptr, s))) return rc;
      }
      break;
    }
    case kPoints:
    case kFlux:
      return GNA_OK;  // configuration tables, computed at bind time
  }
  if ((rc = check_hip(hipGetLastError(), "graph node kernel"))) return rc;
  nd.dev_valid = true;
  nd.host_valid = false;
  return GNA_OK;
}

// The node on its target.  With failover on (off unless the caller asks), a
// GPU node whose launch or copies report a HIP error is computed on the CPU
// instead and the recovery is counted; the node keeps its GPU target.
int compute(gna_graph* g, int id, hipStream_t s) {
  Node& nd = g->nodes[id];
  if (nd.kind == kPoints || nd.kind == kFlux) return GNA_OK;
  if (nd.target == GNA_TARGET_CPU) return compute_cpu(g, id, s);
  int rc = compute_gpu(g, id, s);
  if (rc == GNA_E_HIP && g->failover && has_cpu_form(nd.kind)) {
    ++nd.failovers;
    clear_error();
    rc = compute_cpu(g, id, s);
  }
  return rc;
}

size_t layout(gna_graph* g, bool assign) {
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off = align_up(off + std::max<size_t>(b, 8), 256);
    return at;
  };
  for (auto& ge : g->geoms) {
    const size_t p = take(ge.plan_bytes);
    const size_t r = take((size_t)ge.n_bins * ge.n_bins * 8);
    const size_t pm = ge.need_mixed ? take(ge.plan_mixed_bytes) : 0;
    if (assign) {
      ge.plan_off = p;
      ge.R_off = r;
      ge.plan_mixed_off = pm;
    }
  }
  for (auto& nd : g->nodes) {
    if (nd.kind == kPoints || nd.kind == kFlux) continue;  // live in the plan
    const size_t o = take((size_t)nd.n * 8);
    const size_t a = nd.kind == kChainNode ? take(5 * 8) : 0;
    if (assign) {
      nd.off = o;
      nd.aux_off = a;
    }
  }
  return off;
}

}  // namespace
}  // namespace gna

using namespace gna;

extern "C" int gna_graph_create(gna_graph** graph_out) {
  clear_error();
  if (!graph_out) return fail(GNA_E_INVAL, "gna_graph_create: NULL output");
  *graph_out = new (std::nothrow) gna_graph();
  if (!*graph_out) return fail(GNA_E_INVAL, "gna_graph_create: out of host memory");
  return GNA_OK;
}

extern "C" int gna_graph_destroy(gna_graph* graph) {
  if (!graph) return GNA_OK;
  for (auto& ge : graph->geoms) {
    gna_plan_destroy(ge.plan);
    gna_plan_destroy(ge.plan_mixed);
  }
  if (graph->pinned) (void)hipHostFree(graph->pinned);
  delete graph;
  return GNA_OK;
}

extern "C" int gna_graph_variable(gna_graph* graph, const char* name, double value,
                                  int32_t* var_out) {
  clear_error();
  int rc = creation_open(graph, var_out, "gna_graph_variable");
  if (rc) return rc;
  if (!std::isfinite(value)) return fail(GNA_E_INVAL, "gna_graph_variable: value not finite");
  *var_out = (int32_t)graph->var_value.size();
  graph->var_value.push_back(value);
  graph->var_name.emplace_back(name ? name : "");
  graph->var_users.emplace_back();
  return GNA_OK;
}

extern "C" int gna_graph_points(gna_graph* graph, const gna_model* model,
                                const gna_problem* problem, int32_t* node_out) {
  clear_error();
  int rc = creation_open(graph, node_out, "gna_graph_points");
  if (rc) return rc;
  if (!model || !problem) return fail(GNA_E_INVAL, "gna_graph_points: NULL model or problem");
  size_t bytes = 0;
  // Validates the problem and sizes the configuration plan (host only).
  if ((rc = gna_chain_workspace_size(model, problem, GNA_FP64, 1, nullptr, &bytes))) return rc;
  Geometry ge;
  ge.model = *model;
  ge.edges.assign(problem->edges, problem->edges + problem->n_bins + 1);
  ge.L.assign(problem->L_km, problem->L_km + problem->n_L);
  if (problem->wL) ge.wL.assign(problem->wL, problem->wL + problem->n_L);
  if (problem->data)
    ge.data.assign(problem->data, problem->data + problem->n_bins);
  else
    ge.data.assign(problem->n_bins, 0.0);
  ge.problem = *problem;
  ge.n_bins = problem->n_bins;
  ge.ppb = problem->gl_order * problem->n_sub;
  ge.plan_bytes = bytes;
  const int gid = (int)graph->geoms.size();
  graph->geoms.push_back(std::move(ge));
  Geometry& gr = graph->geoms.back();
  gr.problem.edges = gr.edges.data();
  gr.problem.L_km = gr.L.data();
  gr.problem.wL = gr.wL.empty() ? nullptr : gr.wL.data();
  gr.problem.data = gr.data.data();
  Node nd{};
  nd.kind = kPoints;
  nd.geom = gid;
  nd.n = (int64_t)gr.n_bins * gr.ppb;
  return add_node(graph, std::move(nd), node_out);
}

extern "C" int gna_graph_flux(gna_graph* graph, int32_t points, int32_t* node_out) {
  clear_error();
  int rc = creation_open(graph, node_out, "gna_graph_flux");
  if (rc || (rc = check_node(graph, points, "gna_graph_flux"))) return rc;
  if (graph->nodes[points].kind != kPoints)
    return fail(GNA_E_INVAL, "gna_graph_flux: node %d is not a geometry", points);
  Node nd{};
  nd.kind = kFlux;
  nd.geom = graph->nodes[points].geom;
  nd.n = graph->nodes[points].n;
  nd.inputs = {points};
  return add_node(graph, std::move(nd), node_out);
}

static int check_baseline(double L_km, const char* what) {
  if (!(L_km >= 0.0) || !std::isfinite(L_km)) return fail(GNA_E_INVAL, "%s: L = %g", what, L_km);
  return GNA_OK;
}

extern "C" int gna_graph_oscprob(gna_graph* graph, int32_t energies, double L_km,
                                 const int32_t vars[4], int32_t* node_out) {
  clear_error();
  int rc = creation_open(graph, node_out, "gna_graph_oscprob");
  if (rc || (rc = check_node(graph, energies, "gna_graph_oscprob"))) return rc;
  if (!vars) return fail(GNA_E_INVAL, "gna_graph_oscprob: NULL variables");
  for (int k = 0; k < 4; ++k)
    if ((rc = check_var(graph, vars[k], "gna_graph_oscprob"))) return rc;
  if ((rc = check_baseline(L_km, "gna_graph_oscprob"))) return rc;
  Node nd{};
  nd.kind = kOscProb;
  nd.inputs = {energies};
  nd.vars = {vars[0], vars[1], vars[2], vars[3]};
  nd.L = L_km;
  nd.n = graph->nodes[energies].n;
  return add_node(graph, std::move(nd), node_out);
}

extern "C" int gna_graph_osc_item(gna_graph* graph, int32_t energies, double L_km,
                                  int32_t dm21_var, int32_t dm31_var, int32_t pair, int32_t item,
                                  int32_t* node_out) {
  clear_error();
  int rc = creation_open(graph, node_out, "gna_graph_osc_item");
  if (rc || (rc = check_node(graph, energies, "gna_graph_osc_item")) ||
      (rc = check_var(graph, dm21_var, "gna_graph_osc_item")) ||
      (rc = check_var(graph, dm31_var, "gna_graph_osc_item")) ||
      (rc = check_baseline(L_km, "gna_graph_osc_item")))
    return rc;
  if (pair < 0 || pair > 2) return fail(GNA_E_INVAL, "gna_graph_osc_item: pair %d not 0..2", pair);
  if (item != 0 && item != 1) return fail(GNA_E_INVAL, "gna_graph_osc_item: item %d not 0/1", item);
  Node nd{};
  nd.kind = kOscItem;
  nd.inputs = {energies};
  nd.vars = {dm21_var, dm31_var};  // values read by the node (taints: see below)
  nd.L = L_km;
  nd.pair = pair;
  nd.item = item;
  nd.n = graph->nodes[energies].n;
  const int32_t r = add_node(graph, std::move(nd), node_out);
  if (r) return r;
  // A phase depends only on its own splittings (phi21 on dm2_21, phi31 on
  // dm2_31, phi32 on both): drop the other one from the taint lists.
  const int id = *node_out;
  const int unused = pair == 0 ? dm31_var : (pair == 1 ? dm21_var : -1);
  if (unused >= 0 && dm21_var != dm31_var) {
    auto& users = graph->var_users[unused];
    users.erase(std::remove(users.begin(), users.end(), id), users.end());
  }
  return GNA_OK;
}

static int items_input(gna_graph* graph, const int32_t* items, int k, int want_item,
                       int64_t* n, const char* what) {
  int rc = check_node(graph, items[k], what);
  if (rc) return rc;
  const Node& it = graph->nodes[items[k]];
  if (it.kind != kOscItem || it.pair != k % 3 || it.item != want_item)
    return fail(GNA_E_INVAL, "%s: input %d must be the %s item of pair %d", what, k,
                want_item == 0 ? "sin^2" : "sin 2phi", k % 3);
  if (*n >= 0 && it.n != *n) return fail(GNA_E_INVAL, "%s: items differ in length", what);
  *n = it.n;
  return GNA_OK;
}

extern "C" int gna_graph_pee_items(gna_graph* graph, const int32_t sin2_items[3],
                                   int32_t s12_var, int32_t s13_var, int32_t* node_out) {
  clear_error();
  const char* what = "gna_graph_pee_items";
  int rc = creation_open(graph, node_out, what);
  if (rc || (rc = check_var(graph, s12_var, what)) || (rc = check_var(graph, s13_var, what)))
    return rc;
  if (!sin2_items) return fail(GNA_E_INVAL, "%s: NULL items", what);
  int64_t n = -1;
  for (int k = 0; k < 3; ++k)
    if ((rc = items_input(graph, sin2_items, k, 0, &n, what))) return rc;
  Node nd{};
  nd.kind = kPeeItems;
  nd.inputs = {sin2_items[0], sin2_items[1], sin2_items[2]};
  nd.vars = {s12_var, s13_var};
  nd.n = n;
  return add_node(graph, std::move(nd), node_out);
}

static int check_flavours(int32_t alpha, int32_t beta, int32_t anti, const char* what) {
  if (alpha < 0 || alpha > 2 || beta < 0 || beta > 2)
    return fail(GNA_E_INVAL, "%s: flavours %d -> %d outside 0..2", what, alpha, beta);
  if (anti != 0 && anti != 1) return fail(GNA_E_INVAL, "%s: antineutrino flag %d", what, anti);
  return GNA_OK;
}

extern "C" int gna_graph_prob_items(gna_graph* graph, int32_t alpha, int32_t beta,
                                    int32_t antineutrino, const int32_t angle_vars[4],
                                    const int32_t sin2_items[3], const int32_t sin2phi_items[3],
                                    int32_t* node_out) {
  clear_error();
  const char* what = "gna_graph_prob_items";
  int rc = creation_open(graph, node_out, what);
  if (rc || (rc = check_flavours(alpha, beta, antineutrino, what))) return rc;
  if (!angle_vars || !sin2_items || !sin2phi_items)
    return fail(GNA_E_INVAL, "%s: NULL argument", what);
  for (int k = 0; k < 4; ++k)
    if ((rc = check_var(graph, angle_vars[k], what))) return rc;
  int64_t n = -1;
  int32_t items[6];
  for (int k = 0; k < 3; ++k) {
    items[k] = sin2_items[k];
    items[3 + k] = sin2phi_items[k];
  }
  for (int k = 0; k < 6; ++k)
    if ((rc = items_input(graph, items, k, k < 3 ? 0 : 1, &n, what))) return rc;
  Node nd{};
  nd.kind = kProbItems;
  nd.inputs.assign(items, items + 6);
  nd.vars = {angle_vars[0], angle_vars[1], angle_vars[2], angle_vars[3]};
  nd.alpha = alpha;
  nd.beta = beta;
  nd.anti = antineutrino;
  nd.n = n;
  return add_node(graph, std::move(nd), node_out);
}

extern "C" int gna_graph_prob(gna_graph* graph, int32_t energies, double L_km, int32_t alpha,
                              int32_t beta, int32_t antineutrino, const int32_t angle_vars[4],
                              const int32_t dm_vars[2], int32_t* node_out) {
  clear_error();
  const char* what = "gna_graph_prob";
  int rc = creation_open(graph, node_out, what);
  if (rc || (rc = check_node(graph, energies, what)) ||
      (rc = check_flavours(alpha, beta, antineutrino, what)) ||
      (rc = check_baseline(L_km, what)))
    return rc;
  if (!angle_vars || !dm_vars) return fail(GNA_E_INVAL, "%s: NULL variables", what);
  for (int k = 0; k < 4; ++k)
    if ((rc = check_var(graph, angle_vars[k], what))) return rc;
  for (int k = 0; k < 2; ++k)
    if ((rc = check_var(graph, dm_vars[k], what))) return rc;
  Node nd{};
  nd.kind = kProb;
  nd.inputs = {energies};
  nd.vars = {angle_vars[0], angle_vars[1], angle_vars[2], angle_vars[3], dm_vars[0], dm_vars[1]};
  nd.L = L_km;
  nd.alpha = alpha;
  nd.beta = beta;
  nd.anti = antineutrino;
  nd.n = graph->nodes[energies].n;
  return add_node(graph, std::move(nd), node_out);
}

extern "C" int gna_graph_sum(gna_graph* graph, int32_t n_inputs, const int32_t* inputs,
                             const double* weights, int32_t* node_out) {
  clear_error();
  int rc = creation_open(graph, node_out, "gna_graph_sum");
  if (rc) return rc;
  if (n_inputs < 1 || n_inputs > kMaxSumInputs || !inputs || !weights)
    return fail(GNA_E_INVAL, "gna_graph_sum: %d inputs (1..%d, non-NULL)", n_inputs,
                kMaxSumInputs);
  Node nd{};
  nd.kind = kSum;
  for (int k = 0; k < n_inputs; ++k) {
    if ((rc = check_node(graph, inputs[k], "gna_graph_sum"))) return rc;
    if (graph->nodes[inputs[k]].n != graph->nodes[inputs[0]].n)
      return fail(GNA_E_INVAL, "gna_graph_sum: inputs differ in length");
    if (!std::isfinite(weights[k])) return fail(GNA_E_INVAL, "gna_graph_sum: weight not finite");
    nd.inputs.push_back(inputs[k]);
    nd.w.push_back(weights[k]);
  }
  nd.n = graph->nodes[inputs[0]].n;
  return add_node(graph, std::move(nd), node_out);
}

extern "C" int gna_graph_product(gna_graph* graph, int32_t a, int32_t b, int32_t* node_out) {
  clear_error();
  int rc = creation_open(graph, node_out, "gna_graph_product");
  if (rc || (rc = check_node(graph, a, "gna_graph_product")) ||
      (rc = check_node(graph, b, "gna_graph_product")))
    return rc;
  if (graph->nodes[a].n != graph->nodes[b].n)
    return fail(GNA_E_INVAL, "gna_graph_product: inputs differ in length");
  Node nd{};
  nd.kind = kProduct;
  nd.inputs = {a, b};
  nd.n = graph->nodes[a].n;
  return add_node(graph, std::move(nd), node_out);
}

// A node of a geometry: the input x is per quadrature point (per_point) or
// per bin, the output has n_out elements.
static int per_geometry(gna_graph* graph, NodeKind kind, int32_t x, int32_t points,
                        int per_point, int64_t n_out, int32_t* node_out, const char* what) {
  int rc = creation_open(graph, node_out, what);
  if (rc || (rc = check_node(graph, x, what)) || (rc = check_node(graph, points, what))) return rc;
  if (graph->nodes[points].kind != kPoints)
    return fail(GNA_E_INVAL, "%s: node %d is not a geometry", what, points);
  const Geometry& ge = graph->geoms[graph->nodes[points].geom];
  const int64_t need = per_point ? (int64_t)ge.n_bins * ge.ppb : ge.n_bins;
  if (graph->nodes[x].n != need)
    return fail(GNA_E_INVAL, "%s: input has %lld elements, the geometry needs %lld", what,
                (long long)graph->nodes[x].n, (long long)need);
  Node nd{};
  nd.kind = kind;
  nd.inputs = {x, points};
  nd.geom = graph->nodes[points].geom;
  nd.n = n_out;
  return add_node(graph, std::move(nd), node_out);
}

static int64_t geometry_bins(const gna_graph* graph, int32_t points) {
  if (!graph || points < 0 || points >= (int)graph->nodes.size() ||
      graph->nodes[points].kind != kPoints)
    return 0;  // per_geometry reports the error
  return graph->geoms[graph->nodes[points].geom].n_bins;
}

extern "C" int gna_graph_integrate(gna_graph* graph, int32_t x, int32_t points,
                                   int32_t* node_out) {
  clear_error();
  return per_geometry(graph, kIntegrate, x, points, 1, geometry_bins(graph, points), node_out,
                      "gna_graph_integrate");
}

extern "C" int gna_graph_smear(gna_graph* graph, int32_t x, int32_t points, int32_t* node_out) {
  clear_error();
  return per_geometry(graph, kSmear, x, points, 0, geometry_bins(graph, points), node_out,
                      "gna_graph_smear");
}

extern "C" int gna_graph_chi2(gna_graph* graph, int32_t nu, int32_t points, int32_t* node_out) {
  clear_error();
  return per_geometry(graph, kChi2, nu, points, 0, 1, node_out, "gna_graph_chi2");
}

extern "C" int gna_graph_scale(gna_graph* graph, int32_t x, int32_t var, int32_t* node_out) {
  clear_error();
  int rc = creation_open(graph, node_out, "gna_graph_scale");
  if (rc || (rc = check_node(graph, x, "gna_graph_scale")) ||
      (rc = check_var(graph, var, "gna_graph_scale")))
    return rc;
  Node nd{};
  nd.kind = kScale;
  nd.inputs = {x};
  nd.vars = {var};
  nd.n = graph->nodes[x].n;
  return add_node(graph, std::move(nd), node_out);
}

extern "C" int gna_graph_chain(gna_graph* graph, int32_t points, const int32_t vars[5],
                               int32_t prec, int32_t* node_out) {
  clear_error();
  const char* what = "gna_graph_chain";
  int rc = creation_open(graph, node_out, what);
  if (rc || (rc = check_node(graph, points, what))) return rc;
  if (graph->nodes[points].kind != kPoints)
    return fail(GNA_E_INVAL, "%s: node %d is not a geometry", what, points);
  if (prec != GNA_FP64 && prec != GNA_MIXED) return fail(GNA_E_INVAL, "%s: bad prec %d", what, prec);
  if (!vars) return fail(GNA_E_INVAL, "%s: NULL variables", what);
  for (int k = 0; k < 5; ++k)
    if ((rc = check_var(graph, vars[k], what))) return rc;
  Geometry& ge = graph->geoms[graph->nodes[points].geom];
  if (prec == GNA_MIXED && !ge.need_mixed) {
    size_t bytes = 0;
    if ((rc = gna_chain_workspace_size(&ge.model, &ge.problem, GNA_MIXED, 1, nullptr, &bytes)))
      return rc;
    ge.plan_mixed_bytes = bytes;
    ge.need_mixed = true;
  }
  Node nd{};
  nd.kind = kChainNode;
  nd.inputs = {points};
  nd.vars = {vars[0], vars[1], vars[2], vars[3], vars[4]};
  nd.geom = graph->nodes[points].geom;
  nd.prec = prec;
  nd.n = 6;
  return add_node(graph, std::move(nd), node_out);
}

extern "C" int gna_graph_workspace_size(const gna_graph* graph, size_t* bytes) {
  clear_error();
  if (!graph || !bytes) return fail(GNA_E_INVAL, "gna_graph_workspace_size: NULL argument");
  *bytes = layout(const_cast<gna_graph*>(graph), false);
  return GNA_OK;
}

extern "C" int gna_graph_bind(gna_graph* graph, void* workspace_dev, size_t workspace_bytes,
                              void* stream) {
  clear_error();
  if (!graph) return fail(GNA_E_INVAL, "gna_graph_bind: graph is NULL");
  if (graph->bound) return fail(GNA_E_INVAL, "gna_graph_bind: already bound");
  if (!workspace_dev || ((uintptr_t)workspace_dev & 255))
    return fail(GNA_E_INVAL, "gna_graph_bind: workspace NULL or not 256-byte aligned");
  const size_t need = layout(graph, true);
  if (workspace_bytes < need)
    return fail(GNA_E_WORKSPACE, "gna_graph_bind: workspace %zu bytes, needs %zu",
                workspace_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  // Host mirrors in page-locked memory (configuration stage): a read's
  // device-to-host copy then goes straight to its destination, without the
  // staging a pageable destination needs.
  size_t mirror = 0;
  for (const auto& nd : graph->nodes) mirror += (size_t)nd.n;
  int rc;
  if (!graph->pinned &&
      (rc = check_hip(hipHostMalloc((void**)&graph->pinned, std::max<size_t>(mirror, 1) * 8,
                                    hipHostMallocDefault),
                      "hipHostMalloc (graph host mirrors)")))
    return rc;
  {
    size_t o = 0;
    for (auto& nd : graph->nodes) {
      nd.host = graph->pinned + o;
      o += (size_t)nd.n;
    }
  }
  graph->ws = (unsigned char*)workspace_dev;
  graph->ws_bytes = workspace_bytes;
  for (auto& ge : graph->geoms) {
    // The configuration tables (E_k, f_k, the band of R, data) of a one-point
    // FP64 chain plan; the dense R the smearing node reads is expanded from it.
    if ((rc = gna_chain_create(&ge.model, &ge.problem, GNA_FP64, 1, nullptr,
                               graph->ws + ge.plan_off, ge.plan_bytes, stream, &ge.plan)))
      return rc;
    if ((rc = gna_plan_tables(ge.plan, 0, nullptr, nullptr, (double*)(graph->ws + ge.R_off),
                              stream)))
      return rc;
    if (ge.need_mixed &&
        (rc = gna_chain_create(&ge.model, &ge.problem, GNA_MIXED, 1, nullptr,
                               graph->ws + ge.plan_mixed_off, ge.plan_mixed_bytes, stream,
                               &ge.plan_mixed)))
      return rc;
  }
  for (auto& nd : graph->nodes) {
    if (nd.kind == kPoints || nd.kind == kFlux) {
      const gna_plan* p = graph->geoms[nd.geom].plan;
      nd.table = (const double*)(p->ws + (nd.kind == kPoints ? p->lay.E : p->lay.f));
      nd.dirty = false;
      nd.dev_valid = true;
    }
  }
  if ((rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize (graph bind)"))) return rc;
  graph->bound = true;
  return GNA_OK;
}

extern "C" int gna_graph_set(gna_graph* graph, int32_t var, double value) {
  clear_error();
  if (!graph) return fail(GNA_E_INVAL, "gna_graph_set: graph is NULL");
  int rc = check_var(graph, var, "gna_graph_set");
  if (rc) return rc;
  if (!std::isfinite(value)) return fail(GNA_E_INVAL, "gna_graph_set: value not finite");
  if (graph->var_value[var] == value) return GNA_OK;  // nothing changes
  graph->var_value[var] = value;
  for (int id : graph->var_users[var]) taint(graph, id);
  return GNA_OK;
}

extern "C" int gna_graph_set_target(gna_graph* graph, int32_t node, int32_t target) {
  clear_error();
  if (!graph) return fail(GNA_E_INVAL, "gna_graph_set_target: graph is NULL");
  if (target != GNA_TARGET_GPU && target != GNA_TARGET_CPU)
    return fail(GNA_E_INVAL, "gna_graph_set_target: target %d not GPU (0) or CPU (1)", target);
  if (node == -1) {
    for (auto& nd : graph->nodes)
      if (has_cpu_form(nd.kind)) nd.target = target;
    return GNA_OK;
  }
  int rc = check_node(graph, node, "gna_graph_set_target");
  if (rc) return rc;
  Node& nd = graph->nodes[node];
  if (!has_cpu_form(nd.kind)) {
    if (target == GNA_TARGET_GPU) return GNA_OK;
    return fail(GNA_E_UNSUPPORTED,
                "gna_graph_set_target: node %d (a configuration table or the fused chain) "
                "runs on the GPU only", node);
  }
  nd.target = target;
  return GNA_OK;
}

extern "C" int gna_graph_eval(gna_graph* graph, int32_t node, void* stream, const double** out_dev,
                              int64_t* n_out) {
  clear_error();
  if (!graph) return fail(GNA_E_INVAL, "gna_graph_eval: graph is NULL");
  if (!graph->bound) return fail(GNA_E_INVAL, "gna_graph_eval: graph not bound");
  int rc = check_node(graph, node, "gna_graph_eval");
  hipStream_t s = (hipStream_t)stream;
  if (rc || (rc = evaluate(graph, node, s)) || (rc = ensure_dev(graph, node, s))) return rc;
  if (out_dev) *out_dev = dev_ptr(graph, graph->nodes[node]);
  if (n_out) *n_out = graph->nodes[node].n;
  return GNA_OK;
}

extern "C" int gna_graph_read(gna_graph* graph, int32_t node, double* host_out, int64_t n,
                              void* stream) {
  clear_error();
  if (!graph) return fail(GNA_E_INVAL, "gna_graph_read: graph is NULL");
  if (!graph->bound) return fail(GNA_E_INVAL, "gna_graph_read: graph not bound");
  int rc = check_node(graph, node, "gna_graph_read");
  if (rc) return rc;
  if (!host_out || n != graph->nodes[node].n)
    return fail(GNA_E_INVAL, "gna_graph_read: host buffer of %lld for %lld values", (long long)n,
                (long long)graph->nodes[node].n);
  hipStream_t s = (hipStream_t)stream;
  if ((rc = evaluate(graph, node, s)) || (rc = ensure_host(graph, node, s))) return rc;
  std::memcpy(host_out, graph->nodes[node].host, (size_t)n * 8);
  return GNA_OK;
}

extern "C" int gna_graph_node_info(const gna_graph* graph, int32_t node, int64_t* n_out,
                                   int64_t* evaluations) {
  clear_error();
  if (!graph) return fail(GNA_E_INVAL, "gna_graph_node_info: graph is NULL");
  int rc = check_node(graph, node, "gna_graph_node_info");
  if (rc) return rc;
  if (n_out) *n_out = graph->nodes[node].n;
  if (evaluations) *evaluations = graph->nodes[node].evals;
  return GNA_OK;
}

extern "C" int gna_graph_set_failover(gna_graph* graph, int32_t on) {
  clear_error();
  if (!graph) return fail(GNA_E_INVAL, "gna_graph_set_failover: graph is NULL");
  if (on != 0 && on != 1) return fail(GNA_E_INVAL, "gna_graph_set_failover: %d not 0/1", on);
  graph->failover = on != 0;
  return GNA_OK;
}

extern "C" int gna_graph_node_stats(const gna_graph* graph, int32_t node, int64_t stats[5],
                                    int32_t* target) {
  clear_error();
  if (!graph) return fail(GNA_E_INVAL, "gna_graph_node_stats: graph is NULL");
  int rc = check_node(graph, node, "gna_graph_node_stats");
  if (rc) return rc;
  const Node& nd = graph->nodes[node];
  if (stats) {
    stats[0] = nd.n;
    stats[1] = nd.evals;
    stats[2] = nd.d2h;
    stats[3] = nd.h2d;
    stats[4] = nd.failovers;
  }
  if (target) *target = nd.target;
  return GNA_OK;
}
