// Transformation graph over the kernels (Sec. 2): vector-in / vector-out
// nodes owning their FP64 outputs, scalar variables, a configuration stage
// that places every output in one caller-allocated workspace, and lazy
// evaluation in which changing a variable taints only the nodes that depend
// on it.  Each node runs its own (unfused) kernel, so any intermediate output
// can be read back (Sec. 4.2).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gna_internal.h"
#include "gna_math.h"

namespace gna {
namespace {

enum NodeKind { kPoints, kFlux, kOscProb, kSum, kProduct, kIntegrate, kSmear, kScale, kChi2 };
constexpr int kMaxSumInputs = 64;

struct Geometry {
  gna_model model;
  gna_problem problem;  // pointers below point into the vectors
  std::vector<double> edges, L, wL, data;
  int n_bins = 0, ppb = 0;
  size_t plan_bytes = 0, plan_off = 0, R_off = 0;
  gna_plan* plan = nullptr;
};

struct Node {
  NodeKind kind;
  std::vector<int> inputs;   // node ids
  std::vector<int> vars;     // variable ids
  std::vector<double> w;     // sum weights
  int geom = -1;             // geometry (points-derived nodes)
  double L = 0.0;            // oscprob baseline
  int64_t n = 0;             // output length
  size_t off = 0;            // output offset in the workspace (or table address)
  const double* table = nullptr;  // configuration tables: output lives in a plan
  bool dirty = true;
  int64_t evals = 0;
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

unsigned blocks_for(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

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
  bool bound = false;
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

const double* out_ptr(const gna_graph* g, const Node& nd) {
  return nd.table ? nd.table : (const double*)(g->ws + nd.off);
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

int compute(gna_graph* g, int id, hipStream_t s) {
  Node& nd = g->nodes[id];
  double* out = (double*)(g->ws + nd.off);
  const int t = 256;
  switch (nd.kind) {
    case kPoints:
    case kFlux:
      return GNA_OK;  // configuration tables, computed at bind time
    case kOscProb: {
      const double th[4] = {g->var_value[nd.vars[0]], g->var_value[nd.vars[1]],
                            g->var_value[nd.vars[2]], g->var_value[nd.vars[3]]};
      return gna_pee(out_ptr(g, g->nodes[nd.inputs[0]]), nd.n, 1, &nd.L, nullptr, th, out,
                     GNA_FP64, s);
    }
    case kSum: {
      SumArgs a{};
      a.n_in = (int)nd.inputs.size();
      for (int k = 0; k < a.n_in; ++k) {
        a.x[k] = out_ptr(g, g->nodes[nd.inputs[k]]);
        a.w[k] = nd.w[k];
      }
      hipLaunchKernelGGL(sum_kernel, dim3(blocks_for(nd.n, t)), dim3(t), 0, s, a, nd.n, out);
      break;
    }
    case kProduct:
      hipLaunchKernelGGL(product_kernel, dim3(blocks_for(nd.n, t)), dim3(t), 0, s,
                         out_ptr(g, g->nodes[nd.inputs[0]]), out_ptr(g, g->nodes[nd.inputs[1]]),
                         nd.n, out);
      break;
    case kScale:
      hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(nd.n, t)), dim3(t), 0, s,
                         out_ptr(g, g->nodes[nd.inputs[0]]), g->var_value[nd.vars[0]], nd.n, out);
      break;
    case kIntegrate: {
      const Geometry& ge = g->geoms[nd.geom];
      hipLaunchKernelGGL(integrate_kernel, dim3(blocks_for(ge.n_bins, t)), dim3(t), 0, s,
                         out_ptr(g, g->nodes[nd.inputs[0]]), ge.n_bins, ge.ppb, out);
      break;
    }
    case kSmear: {
      const Geometry& ge = g->geoms[nd.geom];
      const int rows_per_group = t / kWave;
      hipLaunchKernelGGL(smear_kernel, dim3((unsigned)((ge.n_bins + rows_per_group - 1) / rows_per_group)),
                         dim3(t), 0, s, (const double*)(g->ws + ge.R_off),
                         out_ptr(g, g->nodes[nd.inputs[0]]), ge.n_bins, out);
      break;
    }
    case kChi2: {
      const Geometry& ge = g->geoms[nd.geom];
      const double* d = (const double*)(ge.plan->ws + ge.plan->lay.data);
      hipLaunchKernelGGL(chi2_kernel, dim3(1), dim3(1024), 0, s,
                         out_ptr(g, g->nodes[nd.inputs[0]]), d, ge.n_bins, out);
      break;
    }
  }
  return check_hip(hipGetLastError(), "graph node kernel");
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
    if (assign) {
      ge.plan_off = p;
      ge.R_off = r;
    }
  }
  for (auto& nd : g->nodes) {
    if (nd.kind == kPoints || nd.kind == kFlux) continue;  // live in the plan
    const size_t o = take((size_t)nd.n * 8);
    if (assign) nd.off = o;
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
  for (auto& ge : graph->geoms) gna_plan_destroy(ge.plan);
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

extern "C" int gna_graph_oscprob(gna_graph* graph, int32_t energies, double L_km,
                                 const int32_t vars[4], int32_t* node_out) {
  clear_error();
  int rc = creation_open(graph, node_out, "gna_graph_oscprob");
  if (rc || (rc = check_node(graph, energies, "gna_graph_oscprob"))) return rc;
  if (!vars) return fail(GNA_E_INVAL, "gna_graph_oscprob: NULL variables");
  for (int k = 0; k < 4; ++k)
    if ((rc = check_var(graph, vars[k], "gna_graph_oscprob"))) return rc;
  if (!(L_km >= 0.0) || !std::isfinite(L_km))
    return fail(GNA_E_INVAL, "gna_graph_oscprob: L = %g", L_km);
  Node nd{};
  nd.kind = kOscProb;
  nd.inputs = {energies};
  nd.vars = {vars[0], vars[1], vars[2], vars[3]};
  nd.L = L_km;
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
  graph->ws = (unsigned char*)workspace_dev;
  graph->ws_bytes = workspace_bytes;
  int rc;
  for (auto& ge : graph->geoms) {
    // The configuration tables (E_k, f_k, the band of R, data) of a one-point
    // FP64 chain plan; the dense R the smearing node reads is expanded from it.
    if ((rc = gna_chain_create(&ge.model, &ge.problem, GNA_FP64, 1, nullptr,
                               graph->ws + ge.plan_off, ge.plan_bytes, stream, &ge.plan)))
      return rc;
    if ((rc = gna_plan_tables(ge.plan, 0, nullptr, nullptr, (double*)(graph->ws + ge.R_off),
                              stream)))
      return rc;
  }
  for (auto& nd : graph->nodes) {
    if (nd.kind == kPoints || nd.kind == kFlux) {
      const gna_plan* p = graph->geoms[nd.geom].plan;
      nd.table = (const double*)(p->ws + (nd.kind == kPoints ? p->lay.E : p->lay.f));
      nd.dirty = false;
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

extern "C" int gna_graph_eval(gna_graph* graph, int32_t node, void* stream, const double** out_dev,
                              int64_t* n_out) {
  clear_error();
  if (!graph) return fail(GNA_E_INVAL, "gna_graph_eval: graph is NULL");
  if (!graph->bound) return fail(GNA_E_INVAL, "gna_graph_eval: graph not bound");
  int rc = check_node(graph, node, "gna_graph_eval");
  if (rc || (rc = evaluate(graph, node, (hipStream_t)stream))) return rc;
  if (out_dev) *out_dev = out_ptr(graph, graph->nodes[node]);
  if (n_out) *n_out = graph->nodes[node].n;
  return GNA_OK;
}

extern "C" int gna_graph_read(gna_graph* graph, int32_t node, double* host_out, int64_t n,
                              void* stream) {
  clear_error();
  const double* dev = nullptr;
  int64_t len = 0;
  int rc = gna_graph_eval(graph, node, stream, &dev, &len);
  if (rc) return rc;
  if (!host_out || n != len)
    return fail(GNA_E_INVAL, "gna_graph_read: host buffer of %lld for %lld values", (long long)n,
                (long long)len);
  hipStream_t s = (hipStream_t)stream;
  if ((rc = check_hip(hipMemcpyAsync(host_out, dev, (size_t)len * 8, hipMemcpyDeviceToHost, s),
                      "hipMemcpyAsync (graph read)")))
    return rc;
  return check_hip(hipStreamSynchronize(s), "hipStreamSynchronize (graph read)");
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
