// Project-written autotuner for the chain kernels: times each candidate launch
// shape of a plan with HIP events on the caller's stream, keeps the fastest,
// and caches the winner in a small JSON file keyed by the plan's shape bucket,
// precision and GPU architecture.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gna_internal.h"

namespace gna {
namespace {

int bucket(double x) {  // power-of-two bucket
  if (x <= 1) return 0;
  return (int)std::ceil(std::log2(x));
}

std::string cache_key(const gna_plan* p, int B) {
  double ppb = 0, nL = 0, nb = 0, w = 0;
  for (auto& pd : p->probs) {
    ppb += (double)pd.n_bins * pd.ppb;
    nL += (double)pd.n_bins * pd.n_L;
    nb += pd.n_bins;
    w += pd.n_bins;
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s/%s/%s/p%d/nb%d/ppb%d/nL%d/B%d/bins%d", p->arch,
                p->kind == kChain ? "chain" : "fitset", p->prec == GNA_FP64 ? "fp64" : "mixed",
                bucket(p->n_probs), bucket(p->max_bins), bucket(ppb / w), bucket(nL / w),
                bucket(B), bucket(nb));
  return buf;
}

// The cache is a flat JSON object {"key": [threads, G, C, persistent, mfma], ...}.
bool cache_lookup(const char* path, const std::string& key, Shape& sh) {
  FILE* fp = std::fopen(path, "r");
  if (!fp) return false;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), fp)) > 0) text.append(buf, n);
  std::fclose(fp);
  const std::string needle = "\"" + key + "\"";
  const size_t at = text.find(needle);
  if (at == std::string::npos) return false;
  const size_t lb = text.find('[', at);
  if (lb == std::string::npos) return false;
  int v[7] = {0, 0, 0, 0, 0, 1, 0};
  const int got = std::sscanf(text.c_str() + lb, "[%d, %d, %d, %d, %d, %d, %d]", &v[0], &v[1], &v[2],
                              &v[3], &v[4], &v[5], &v[6]);
  // Entries without the sixth value predate phase sharing, without the
  // seventh the split tail.
  if (got < 5) return false;
  sh.threads = v[0];
  sh.G = v[1];
  sh.C = v[2];
  sh.persistent = v[3];
  sh.mfma = v[4];
  sh.share = v[5];
  sh.split = v[6];
  return true;
}

void cache_store(const char* path, const std::string& key, const Shape& sh) {
  std::vector<std::pair<std::string, std::string>> entries;
  if (FILE* fp = std::fopen(path, "r")) {
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), fp)) > 0) text.append(buf, n);
    std::fclose(fp);
    size_t pos = 0;
    while (true) {
      const size_t q0 = text.find('"', pos);
      if (q0 == std::string::npos) break;
      const size_t q1 = text.find('"', q0 + 1);
      const size_t lb = text.find('[', q1);
      const size_t rb = text.find(']', lb);
      if (q1 == std::string::npos || lb == std::string::npos || rb == std::string::npos) break;
      entries.emplace_back(text.substr(q0 + 1, q1 - q0 - 1), text.substr(lb, rb - lb + 1));
      pos = rb + 1;
    }
  }
  char val[96];
  std::snprintf(val, sizeof(val), "[%d, %d, %d, %d, %d, %d, %d]", sh.threads, sh.G, sh.C,
                sh.persistent, sh.mfma, sh.share, sh.split);
  bool found = false;
  for (auto& e : entries)
    if (e.first == key) {
      e.second = val;
      found = true;
    }
  if (!found) entries.emplace_back(key, val);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fp = std::fopen(tmp.c_str(), "w");
  if (!fp) return;
  std::fprintf(fp, "{\n");
  for (size_t i = 0; i < entries.size(); ++i)
    std::fprintf(fp, "  \"%s\": %s%s\n", entries[i].first.c_str(), entries[i].second.c_str(),
                 i + 1 < entries.size() ? "," : "");
  std::fprintf(fp, "}\n");
  std::fclose(fp);
  std::rename(tmp.c_str(), path);
}

int eval_once(gna_plan* p, const double* params, int32_t B, double* chi2, double* grad,
              hipStream_t s) {
  if (p->shape.mfma) return launch_scan(p, params, B, chi2, grad, nullptr, s);
  return launch_chain(p, params, B, chi2, grad, nullptr, s);
}

}  // namespace
}  // namespace gna

using namespace gna;

extern "C" int gna_plan_autotune(gna_plan* plan, const double* params_dev, int32_t B,
                                 double* chi2_dev, double* grad_dev, int32_t reps,
                                 const char* cache_path, void* stream, int32_t shape_out[7]) {
  clear_error();
  if (!plan || !plan->ws) return fail(GNA_E_INVAL, "plan is NULL");
  if (!params_dev || !chi2_dev) return fail(GNA_E_INVAL, "params or chi2 NULL");
  if (plan->kind == kFitset) B = plan->n_points;
  if (B < 1 || B > plan->n_points) return fail(GNA_E_INVAL, "B = %d out of range", B);
  if (reps < 1) reps = 10;
  hipStream_t s = (hipStream_t)stream;
  const std::string key = cache_key(plan, B);
  Shape best = plan->shape;
  int rc;
  if (cache_path && cache_lookup(cache_path, key, best)) {
    rc = apply_shape(plan, best, s);
    if (rc == GNA_OK) {
      if (shape_out) gna_plan_shape(plan, shape_out, nullptr);
      return GNA_OK;
    }
  }
  const std::vector<Shape> cands = shape_candidates(plan);
  hipEvent_t e0, e1;
  if ((rc = check_hip(hipEventCreate(&e0), "hipEventCreate"))) return rc;
  if ((rc = check_hip(hipEventCreate(&e1), "hipEventCreate"))) {
    (void)hipEventDestroy(e0);
    return rc;
  }
  double best_ms = 1e300;
  Shape start = plan->shape;
  for (const Shape& c : cands) {
    if (apply_shape(plan, c, s) != GNA_OK) continue;
    if (eval_once(plan, params_dev, B, chi2_dev, grad_dev, s) != GNA_OK) continue;  // warm-up
    std::vector<float> t;
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) {
      ok = hipEventRecord(e0, s) == hipSuccess &&
           eval_once(plan, params_dev, B, chi2_dev, grad_dev, s) == GNA_OK &&
           hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
      float ms = 0;
      if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) t.push_back(ms);
    }
    if (!ok || t.empty()) continue;
    std::nth_element(t.begin(), t.begin() + t.size() / 2, t.end());
    const double med = t[t.size() / 2];
    if (med < best_ms) {
      best_ms = med;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_ms >= 1e300) best = start;
  if ((rc = apply_shape(plan, best, s))) return rc;
  if (cache_path) cache_store(cache_path, key, best);
  if (shape_out) gna_plan_shape(plan, shape_out, nullptr);
  clear_error();
  return GNA_OK;
}
