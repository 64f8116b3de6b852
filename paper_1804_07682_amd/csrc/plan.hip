// Configuration stage of the chain (Sec. 2: the graph is configured once and
// evaluated many times; Sec. 4.2: every buffer is allocated at configuration).
//
// Host side: validation, the workspace layout, the band structure of the
// smearing matrix, the tile list of an uneven batch.  Device side: kernels
// that build the Gauss-Legendre rules, the quadrature energies E_k, the
// flux factors f_k = n0 w_k S(E_k) sigma(E_k) and the banded smearing matrix.
#include <algorithm>
#include <deque>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>

#include "gna_internal.h"
#include "gna_math.h"

namespace gna {
namespace {

// ---------------------------------------------------------------------------
// Gauss-Legendre rules of orders 1..64, rule n stored at n(n-1)/2, nodes
// ascending.  Newton's method on the Legendre polynomial P_n (three-term
// recurrence, P_n' = n (x P_n - P_{n-1}) / (x^2 - 1)) from the start
// cos(pi (i - 1/4) / (n + 1/2)); weights 2 / ((1 - x^2) P_n'(x)^2).
// One work-group per order, one lane per root of the positive half.
// ---------------------------------------------------------------------------
__device__ void legendre_pair(int n, double x, double& pn, double& pnm1) {
  double a = 1.0, b = x;  // P_0, P_1
  for (int k = 1; k < n; ++k) {
    const double c = ((2.0 * k + 1.0) * x * b - k * a) / (k + 1.0);
    a = b;
    b = c;
  }
  pn = (n == 0) ? 1.0 : b;
  pnm1 = (n == 0) ? 0.0 : a;
}

// Rule of order n into t[0..n), w[0..n); lanes 0..31 of the calling group.
__device__ void gl_rule(int n, double* __restrict__ t, double* __restrict__ w) {
  const int i = threadIdx.x + 1;  // root index from the top
  const double pi = 3.14159265358979323846;
  if (i <= n / 2) {
    double x = cos(pi * (i - 0.25) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pn, pm;
      legendre_pair(n, x, pn, pm);
      const double dp = n * (x * pn - pm) / (x * x - 1.0);
      const double dx = pn / dp;
      x = x - dx;
      if (fabs(dx) <= 1e-17) break;
    }
    double pn, pm;
    legendre_pair(n, x, pn, pm);
    const double dp = n * (x * pn - pm) / (x * x - 1.0);
    const double wi = 2.0 / ((1.0 - x * x) * dp * dp);
    t[n - i] = x;
    w[n - i] = wi;
    t[i - 1] = -x;
    w[i - 1] = wi;
  }
  if ((n & 1) && threadIdx.x == 0) {
    double pn, pm;
    legendre_pair(n, 0.0, pn, pm);
    const double dp = n * pm;  // n (0 * P_n - P_{n-1}) / (0 - 1)
    t[n / 2] = 0.0;
    w[n / 2] = 2.0 / (dp * dp);
  }
}

__global__ void gl_table_kernel(double* __restrict__ t, double* __restrict__ w) {
  const int n = blockIdx.x + 1;
  const int base = n * (n - 1) / 2;
  gl_rule(n, t + base, w + base);
}

__global__ void gl_one_kernel(int n, double* __restrict__ t, double* __restrict__ w) {
  gl_rule(n, t, w);
}

// Staging of the host-output rule (gna_gl_nodes): nodes, then weights.
static __device__ double gl_stage[2 * kMaxOrder];

__global__ void gl_stage_kernel(int n) { gl_rule(n, gl_stage, gl_stage + kMaxOrder); }

// ---------------------------------------------------------------------------
// Quadrature energies and flux factors, one lane per point (grid.y = problem).
// Point k of a problem: bin j = k / ppb, sub-interval s, node i; on the
// sub-interval [a, b]: E = (a + b)/2 + ((b - a)/2) t_i, w = ((b - a)/2) w_i.
// ---------------------------------------------------------------------------
template <class R>
__global__ void quad_kernel(const ProbDev* __restrict__ probs, const double* __restrict__ edges,
                            const double* __restrict__ glt, const double* __restrict__ glw,
                            gna_model m, double* __restrict__ Eout, R* __restrict__ fout) {
  const ProbDev pd = probs[blockIdx.y];
  const int64_t npts = (int64_t)pd.n_bins * pd.ppb;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npts) return;
  const int j = (int)(k / pd.ppb);
  const int rem = (int)(k - (int64_t)j * pd.ppb);
  const int s = rem / pd.order;
  const int i = rem - s * pd.order;
  const double* e = edges + pd.edge_off;
  const double lo = e[j], hi = e[j + 1];
  const double width = hi - lo;
  const double a = lo + (width * s) / pd.n_sub;
  const double b = (s + 1 == pd.n_sub) ? hi : lo + (width * (s + 1)) / pd.n_sub;
  const double c = 0.5 * (a + b);
  const double h = 0.5 * (b - a);
  const int gl = pd.order * (pd.order - 1) / 2;
  const double E = c + h * glt[gl + i];
  const double wk = h * glw[gl + i];
  // Spectrum exp(a0 + a1 E + a2 E^2 + a3 E^3) and IBD cross section.
  const double S = exp(m.spec[0] + m.spec[1] * E + m.spec[2] * E * E + m.spec[3] * E * E * E);
  const double x = E - m.xsec_delta;
  const double sig = (x <= m.m_e) ? 0.0 : x * sqrt(x * x - m.m_e * m.m_e);
  Eout[pd.pt_off + k] = E;
  fout[pd.pt_off + k] = (R)(m.n0 * wk * S * sig);
}

// ---------------------------------------------------------------------------
// Banded smearing matrix: one work-group (64 lanes) per 64-row slice, looping
// over its diagonals.  R_ij = (erf((e_{i+1} - Ebar_j)/(sqrt2 s_j))
//                            - erf((e_i - Ebar_j)/(sqrt2 s_j))) / 2,
// Ebar_j the centre of bin j, s_j = res_a sqrt(Ebar_j).  Entries outside the
// matrix are stored as 0.
// ---------------------------------------------------------------------------
template <class R>
__global__ void band_kernel(const ProbDev* __restrict__ probs, const SliceDev* __restrict__ slices,
                            const int32_t* __restrict__ slice_prob,
                            const double* __restrict__ edges, double res_a, R* __restrict__ Rv) {
  const int64_t gs = blockIdx.x;
  const int p = slice_prob[gs];
  const ProbDev pd = probs[p];
  const SliceDev sd = slices[gs];
  const int s = (int)(gs - pd.slice_off);
  const int i = s * kSlice + (int)threadIdx.x;
  const double* e = edges + pd.edge_off;
  const double sqrt2 = 1.4142135623730951;
  for (int dd = 0; dd < sd.nd; ++dd) {
    const int j = i + sd.dlo + dd;
    double v = 0.0;
    if (i < pd.n_bins && j >= 0 && j < pd.n_bins) {
      const double ebar = 0.5 * (e[j] + e[j + 1]);
      const double sig = res_a * sqrt(ebar);
      const double den = sqrt2 * sig;
      v = 0.5 * (erf((e[i + 1] - ebar) / den) - erf((e[i] - ebar) / den));
    }
    Rv[sd.off + (int64_t)dd * kSlice + threadIdx.x] = (R)v;
  }
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <class R>
__global__ void widen_kernel(const R* __restrict__ in, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (double)in[i];
}

// Dense expansion of one problem's band (row i = reconstructed bin).
template <class R>
__global__ void dense_kernel(const ProbDev* __restrict__ probs, int prob,
                             const SliceDev* __restrict__ slices, const R* __restrict__ Rv,
                             double* __restrict__ out) {
  const ProbDev pd = probs[prob];
  const int64_t nb = pd.n_bins;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * nb) return;
  const int i = (int)(idx / nb), j = (int)(idx - (idx / nb) * nb);
  const int s = i / kSlice, l = i - s * kSlice;
  const SliceDev sd = slices[pd.slice_off + s];
  const int d = j - i;
  double v = 0.0;
  if (d >= sd.dlo && d < sd.dlo + sd.nd) v = (double)Rv[sd.off + (int64_t)(d - sd.dlo) * kSlice + l];
  out[idx] = v;
}

// ---------------------------------------------------------------------------
// Host helpers.
// ---------------------------------------------------------------------------
int validate_model(const gna_model* m) {
  if (!m) return fail(GNA_E_INVAL, "model is NULL");
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(m->spec[i])) return fail(GNA_E_INVAL, "model.spec[%d] not finite", i);
  if (!std::isfinite(m->xsec_delta) || !std::isfinite(m->m_e) || !(m->m_e >= 0.0))
    return fail(GNA_E_INVAL, "model cross-section constants invalid");
  if (!std::isfinite(m->n0)) return fail(GNA_E_INVAL, "model.n0 not finite");
  if (!(m->res_a >= 0.0) || !std::isfinite(m->res_a))
    return fail(GNA_E_INVAL, "model.res_a must be finite and >= 0");
  return GNA_OK;
}

int validate_problem(const gna_problem* p, int idx) {
  if (!p) return fail(GNA_E_INVAL, "problem %d is NULL", idx);
  if (p->n_bins < 1 || p->n_bins > kMaxBins)
    return fail(GNA_E_INVAL, "problem %d: n_bins = %d outside 1..%d", idx, p->n_bins, kMaxBins);
  if (!p->edges) return fail(GNA_E_INVAL, "problem %d: edges NULL", idx);
  for (int j = 0; j <= p->n_bins; ++j)
    if (!std::isfinite(p->edges[j]) || !(p->edges[j] > 0.0))
      return fail(GNA_E_INVAL, "problem %d: edge %d = %g must be finite and > 0", idx, j,
                  p->edges[j]);
  for (int j = 0; j < p->n_bins; ++j)
    if (!(p->edges[j + 1] > p->edges[j]))
      return fail(GNA_E_INVAL, "problem %d: edges not strictly increasing at %d", idx, j);
  if (p->gl_order < 1 || p->gl_order > kMaxOrder)
    return fail(GNA_E_INVAL, "problem %d: gl_order = %d outside 1..%d", idx, p->gl_order,
                kMaxOrder);
  if (p->n_sub < 1 || (int64_t)p->n_sub * p->gl_order > kMaxPPB)
    return fail(GNA_E_INVAL, "problem %d: n_sub = %d invalid", idx, p->n_sub);
  if (p->n_L < 1 || p->n_L > kMaxBaselines)
    return fail(GNA_E_INVAL, "problem %d: n_L = %d outside 1..%d", idx, p->n_L, kMaxBaselines);
  if (!p->L_km) return fail(GNA_E_INVAL, "problem %d: L_km NULL", idx);
  for (int r = 0; r < p->n_L; ++r) {
    if (!std::isfinite(p->L_km[r]) || !(p->L_km[r] >= 0.0))
      return fail(GNA_E_INVAL, "problem %d: L[%d] = %g invalid", idx, r, p->L_km[r]);
    if (p->wL && !std::isfinite(p->wL[r]))
      return fail(GNA_E_INVAL, "problem %d: wL[%d] not finite", idx, r);
  }
  if (!p->data) return fail(GNA_E_INVAL, "problem %d: data NULL", idx);
  for (int j = 0; j < p->n_bins; ++j)
    if (!(p->data[j] >= 0.0) || !std::isfinite(p->data[j]))
      return fail(GNA_E_INVAL, "problem %d: data[%d] = %g must be finite and >= 0", idx, j,
                  p->data[j]);
  return GNA_OK;
}

// Row band of column j: rows i with e_i < Ebar_j + Z sqrt2 s_j and
// e_{i+1} > Ebar_j - Z sqrt2 s_j; outside it both erf arguments exceed
// |z| = 6 with the same sign and R_ij is 0 (to < 1e-17).
void column_band(const double* e, int nb, int j, double res_a, int& ilo, int& ihi) {
  const double ebar = 0.5 * (e[j] + e[j + 1]);
  const double half = kBandZ * 1.4142135623730951 * (res_a * std::sqrt(ebar));
  const double top = ebar + half, bot = ebar - half;
  // first i with e_{i+1} > bot
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    if (e[mid + 1] > bot) hi = mid; else lo = mid + 1;
  }
  ilo = std::min(lo, j);
  // last i with e_i < top
  lo = 0;
  hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (e[mid] < top) lo = mid; else hi = mid - 1;
  }
  ihi = std::max(lo, j);
}

// Slices (dlo, nd) of one problem; returns the number of stored entries.
int64_t build_slices(const double* e, int nb, double res_a, std::vector<SliceDev>& out) {
  const int ns = (nb + kSlice - 1) / kSlice;
  std::vector<int> dmin(ns, 1 << 30), dmax(ns, -(1 << 30));
  for (int j = 0; j < nb; ++j) {
    int ilo, ihi;
    column_band(e, nb, j, res_a, ilo, ihi);
    for (int s = ilo / kSlice; s <= ihi / kSlice; ++s) {
      const int r0 = std::max(ilo, s * kSlice), r1 = std::min(ihi, s * kSlice + kSlice - 1);
      dmin[s] = std::min(dmin[s], j - r1);
      dmax[s] = std::max(dmax[s], j - r0);
    }
  }
  int64_t total = 0;
  for (int s = 0; s < ns; ++s) {
    SliceDev sd{};
    if (dmax[s] < dmin[s]) {  // cannot happen (the diagonal is always in band)
      dmin[s] = 0;
      dmax[s] = 0;
    }
    sd.dlo = dmin[s];
    sd.nd = dmax[s] - dmin[s] + 1;
    sd.off = total;  // relative; made absolute by the caller
    total += (int64_t)sd.nd * kSlice;
    out.push_back(sd);
  }
  return total;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch shapes.
// ---------------------------------------------------------------------------
// LDS of the generic kernel's tail: the point's five vectors when they fit
// the budget (else they stay in the scratch region), then the partial sums
// of up to eight diagonal chunks per slice when those fit too (a chunk of
// each slice per wavefront: at most 5 x threads values), and the per-wave
// reduction slots and flag.
ChainLds chain_lds(const gna_plan* p, const Shape& sh) {
  const size_t rs = (p->prec == GNA_FP64) ? 8 : 4;
  const size_t red = align_up((size_t)(sh.threads / kWave) * 6 * 8, 16) + 16;
  const size_t vec = align_up((size_t)5 * p->max_bins * rs, 16);
  const size_t part = align_up((size_t)5 * sh.threads * rs, 16);
  ChainLds c;
  c.vs = (vec + red <= p->lds_limit) ? p->max_bins : 0;
  const size_t base = (c.vs ? vec : 0) + red;
  c.kf_cap = (base + part <= p->lds_limit) ? 8 : 1;
  c.bytes = base + (c.kf_cap > 1 ? part : 0);
  return c;
}

size_t shape_lds_limit(const gna_plan* p, const Shape& sh) {
  // The queued-tail kernel asks for its LDS at launch (up to the device's
  // per-work-group limit); the generic kernel stays within 64 KB.
  return sh.split == 2 ? p->lds_device : p->lds_limit;
}

size_t chain_lds_bytes(const gna_plan* p, const Shape& sh) {
  if (sh.split == 1) return 0;  // the point pass alone keeps nothing in LDS
  if (sh.split == 2) return queued_lds_bytes(p, sh);  // the tail items' windows
  return chain_lds(p, sh).bytes;
}

namespace {

// Mean work of a problem: points per bin and baselines.
void mean_work(const gna_plan* p, double& ppb, double& nL) {
  double sp = 0, sl = 0, w = 0;
  for (auto& pd : p->probs) {
    const double wt = (double)pd.n_bins;
    sp += wt * pd.ppb;
    sl += wt * pd.n_L;
    w += wt;
  }
  ppb = sp / w;
  nL = sl / w;
}

Shape auto_shape(const gna_plan* p) {
  Shape sh;
  sh.threads = 256;
  double ppb, nL;
  mean_work(p, ppb, nL);
  // Lanes per bin: grow while each lane keeps >= 2 points and >= 16 evaluations.
  int G = 1;
  while (G < 64 && ppb / (2.0 * G) >= 2.0 && ppb * nL / (2.0 * G) >= 16.0) G *= 2;
  sh.G = G;
  const int bpt = sh.threads / G;
  if (p->kind == kChain) {
    const int nb = p->probs[0].n_bins;
    const int nbb = (nb + bpt - 1) / bpt;
    const int64_t blocks = (int64_t)p->n_points * nbb;
    int cmax = (int)std::max(1.0, std::min(ppb / G, ppb * nL / (8.0 * G)));
    cmax = std::min(cmax, p->ccap);
    const int want = (int)std::min<int64_t>(1 << 20, (2048 + blocks - 1) / blocks);
    sh.C = std::max(1, std::min(want, cmax));
  } else {
    sh.C = 1;
    sh.split = 1;
  }
  sh.persistent = 0;
  sh.mfma = 0;
  return sh;
}

}  // namespace

std::vector<Shape> shape_candidates(const gna_plan* p) {
  std::vector<Shape> out;
  const int threads[] = {64, 128, 256, 512, 1024};
  const int Gs[] = {1, 2, 4, 8, 16, 32, 64};
  const int Cs[] = {1, 2, 4, 8, 16, 32, 64};
  double ppb, nL;
  mean_work(p, ppb, nL);
  for (int t : threads)
    for (int G : Gs) {
      if (G > t || G > 2 * ppb) continue;
      if (p->kind == kFitset && t / G < 4) continue;
      for (int C : Cs) {
        // Beyond one point per lane the lanes split (point, baseline) items.
        if (C > p->ccap || C > ppb * nL / G + 1) continue;
        for (int pers = 0; pers <= 1; ++pers)
          for (int split = 0; split <= (p->kind == kFitset ? 2 : 1); ++split) {
            if (split == 2 && !pers) continue;  // the queued tail is a persistent launch
            Shape sh;
            sh.threads = t;
            sh.G = G;
            sh.C = C;
            sh.persistent = pers;
            sh.mfma = 0;
            sh.split = split;
            if (p->tail_pin && split != p->tail_pin - 1) continue;  // the caller chose the tail
            if (chain_lds_bytes(p, sh) > shape_lds_limit(p, sh)) continue;
            out.push_back(sh);
          }
      }
    }
  if (p->kind == kChain && scan_supported(p)) {
    for (int v = 1; v <= 3; ++v)
      for (int share = p->share_allowed; share >= 0; --share) {
        Shape sh;
        sh.mfma = v;
        sh.share = share;
        out.push_back(sh);
      }
  }
  return out;
}

// Queue of the queued tail: the point tiles with one tail item per fit.  The
// fits go in order of falling tail work (the band diagonals of their slices),
// each fit's tiles longest first; a fit's tail item is placed once about one
// turnover of the resident work-groups (kQueuedLagWaves wavefronts per CU) of
// entries has followed its last tile, ahead of later tiles.  So a tail's wait
// for its fit's tiles is short, the tails' band reads overlap the arithmetic
// of later tiles, the longest tails start early, and every tile a tail waits
// for was handed out before it, to a work-group that waits on nothing.
template <class TileAt>
int queued_order(const gna_plan* p, const Shape& sh, size_t n_items, TileAt tile_at,
                 std::vector<TileDev>& tiles, std::vector<int32_t>& qitems) {
  const int nf = (int)p->probs.size();
  const int nw = sh.threads / kWave;
  std::vector<std::vector<size_t>> of_fit(nf);
  for (size_t k = 0; k < n_items; ++k) of_fit[tile_at(k).point].push_back(k);  // longest first
  std::vector<double> tail(nf, 0.0);
  for (size_t i = 0; i < p->slices.size(); ++i) tail[p->slice_prob_host[i]] += p->slices[i].nd;
  std::vector<int> fits(nf);
  for (int f = 0; f < nf; ++f) fits[f] = f;
  std::stable_sort(fits.begin(), fits.end(), [&](int a, int b) { return tail[a] > tail[b]; });
  const int64_t lag = std::max<int64_t>(1, (int64_t)kQueuedLagWaves * p->cu_count / nw);
  std::deque<std::pair<int, int64_t>> ready;  // (fit, first queue position allowed)
  auto emit_ready = [&](bool all) {
    while (!ready.empty() && (all || ready.front().second <= (int64_t)qitems.size())) {
      qitems.push_back(-1 - ready.front().first);
      ready.pop_front();
    }
  };
  for (int f : fits) {
    for (size_t k : of_fit[f]) {
      emit_ready(false);
      qitems.push_back((int32_t)tiles.size());
      tiles.push_back(tile_at(k));
    }
    ready.emplace_back(f, (int64_t)qitems.size() + lag);
  }
  emit_ready(true);
  // A tail's wait ends only if all of its fit's tiles sit earlier in the
  // queue: check that, and that each tile and each fit's tail appears once.
  std::vector<size_t> tiles_seen(nf, 0);
  std::vector<char> tail_seen(nf, 0);
  int64_t n_t = 0, n_f = 0;
  for (int32_t e : qitems) {
    if (e >= 0) {
      if (e != n_t++) return fail(GNA_E_INVAL, "queued tail: tile %d out of order", e);
      ++tiles_seen[tiles[e].point];
      continue;
    }
    const int f = -1 - e;
    if (f >= nf || tail_seen[f] || tiles_seen[f] != of_fit[f].size())
      return fail(GNA_E_INVAL, "queued tail: fit %d queued twice or before its tiles", f);
    tail_seen[f] = 1;
    ++n_f;
  }
  if (n_t != (int64_t)n_items || n_f != nf)
    return fail(GNA_E_INVAL, "queued tail: %lld tiles, %lld fits queued", (long long)n_t,
                (long long)n_f);
  return GNA_OK;
}

int apply_shape(gna_plan* p, const Shape& sh, hipStream_t s) {
  if (sh.threads < kWave || sh.threads > 1024 || (sh.threads & (sh.threads - 1)))
    return fail(GNA_E_INVAL, "threads = %d invalid", sh.threads);
  if (sh.G < 1 || sh.G > kWave || (sh.G & (sh.G - 1)) || sh.G > sh.threads)
    return fail(GNA_E_INVAL, "lanes_per_bin = %d invalid", sh.G);
  if (sh.C < 1) return fail(GNA_E_INVAL, "chunks = %d invalid", sh.C);
  if (sh.split == 2 && p->kind != kFitset)
    return fail(GNA_E_UNSUPPORTED, "a queued tail needs a fitset plan");
  if (sh.split == 2 && !sh.persistent)
    return fail(GNA_E_UNSUPPORTED, "a queued tail needs the persistent launch");
  if (sh.mfma && !(p->kind == kChain && scan_supported(p)))
    return fail(GNA_E_UNSUPPORTED, "MFMA smearing needs a chain plan with n_bins <= 256");
  if (!sh.mfma && chain_lds_bytes(p, sh) > shape_lds_limit(p, sh))
    return fail(GNA_E_UNSUPPORTED, "shape needs %zu bytes of LDS (limit %zu)",
                chain_lds_bytes(p, sh), shape_lds_limit(p, sh));
  std::vector<TileDev> tiles;
  std::vector<int32_t> qitems;
  for (size_t i = 0; i < p->probs.size(); ++i) {
    ProbDev& pd = p->probs[i];
    pd.G = sh.G;
    pd.bins_per_tile = sh.threads / sh.G;
    pd.n_bin_blocks = (pd.n_bins + pd.bins_per_tile - 1) / pd.bins_per_tile;
    // With fewer than two points per lane and several baselines, lanes and
    // chunks take (point, baseline) items instead of whole points.
    pd.by_item = (pd.n_L > 1 && (int64_t)pd.ppb < 2LL * sh.G * sh.C) ? 1 : 0;
    const int units = pd.by_item ? pd.ppb * pd.n_L : pd.ppb;
    pd.C = std::max(1, std::min(std::min(sh.C, units), p->ccap));
  }
  if (p->kind == kChain) {
    p->n_tiles = (int64_t)p->probs[0].n_bin_blocks * p->probs[0].C;
  } else {
    struct Item {
      TileDev t;
      double cost;
    };
    std::vector<Item> items;
    for (size_t i = 0; i < p->probs.size(); ++i) {
      const ProbDev& pd = p->probs[i];
      for (int bb = 0; bb < pd.n_bin_blocks; ++bb) {
        const int nbins = std::min(pd.bins_per_tile, pd.n_bins - bb * pd.bins_per_tile);
        for (int c = 0; c < pd.C; ++c) {
          const int units = pd.by_item ? pd.ppb * pd.n_L : pd.ppb;
          const int k0 = (int)((int64_t)c * units / pd.C);
          const int k1 = (int)((int64_t)(c + 1) * units / pd.C);
          // Lanes of one bin share its points (or items): the tile lasts
          // ceil(units / G) trips of n_L (or one) evaluations.
          const double trips = std::ceil((double)(k1 - k0) / pd.G);
          Item it;
          it.t = TileDev{(int32_t)i, (int32_t)i, bb, c};
          it.cost = trips * (pd.by_item ? 1 : pd.n_L) + 1e-6 * nbins;
          items.push_back(it);
        }
      }
    }
    if ((int64_t)items.size() > p->tile_capacity)
      return fail(GNA_E_UNSUPPORTED, "shape needs %zu tiles, capacity %lld", items.size(),
                  (long long)p->tile_capacity);
    // Longest-processing-time order: the queue hands out the costliest tiles first.
    std::stable_sort(items.begin(), items.end(),
                     [](const Item& a, const Item& b) { return a.cost > b.cost; });
    if (sh.split != 2) {
      for (auto& it : items) tiles.push_back(it.t);
    } else {
      const int rc =
          queued_order(p, sh, items.size(), [&](size_t k) { return items[k].t; }, tiles, qitems);
      if (rc) return rc;
    }
    p->n_tiles = (int64_t)tiles.size();
  }
  p->n_qitems = (int64_t)qitems.size();
  p->shape = sh;
  p->share_phases = p->share_allowed && sh.share;
  p->launch_cache[0].ready = p->launch_cache[1].ready = 0;
  if (p->ws) {
    int rc = check_hip(hipMemcpyAsync(p->ws + p->lay.probs, p->probs.data(),
                                      sizeof(ProbDev) * p->probs.size(), hipMemcpyHostToDevice, s),
                       "hipMemcpyAsync (problem descriptors)");
    if (rc) return rc;
    if (!tiles.empty()) {
      rc = check_hip(hipMemcpyAsync(p->ws + p->lay.tiles, tiles.data(),
                                    sizeof(TileDev) * tiles.size(), hipMemcpyHostToDevice, s),
                     "hipMemcpyAsync (tile list)");
      if (rc) return rc;
    }
    if (!qitems.empty()) {
      rc = check_hip(hipMemcpyAsync(p->ws + p->lay.q_items, qitems.data(), 4 * qitems.size(),
                                    hipMemcpyHostToDevice, s),
                     "hipMemcpyAsync (queue)");
      if (rc) return rc;
    }
    // The host vectors die here: finish the copies first.
    rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize (shape upload)");
    if (rc) return rc;
  }
  return GNA_OK;
}

// ---------------------------------------------------------------------------
// Plan construction shared by chain and fitset plans.
// ---------------------------------------------------------------------------
namespace {

struct PlanBuild {
  gna_plan* p = nullptr;
  std::vector<double> L, wL, edges, data;
  std::vector<int32_t> slice_prob;
};

void compute_layout(gna_plan* p, PlanBuild& b) {
  Layout& L = p->lay;
  const size_t rs = (p->prec == GNA_FP64) ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + std::max<size_t>(bytes, 1), 256);
    return at;
  };
  L.probs = take(sizeof(ProbDev) * p->n_probs);
  L.slices = take(sizeof(SliceDev) * p->total_slices);
  L.slice_prob = take(4 * p->total_slices);
  L.tiles = take(sizeof(TileDev) * std::max<int64_t>(p->tile_capacity, 1));
  L.E = take(8 * p->total_pts);
  L.f = take(rs * p->total_pts);
  L.L = take(8 * b.L.size());
  L.wL = take(8 * b.L.size());
  L.edges = take(8 * b.edges.size());
  L.data = take(8 * b.data.size());
  L.gl = take(16 * kGLTable);
  L.Rv = take(rs * p->total_band);
  L.scratch = take(rs * p->scratch_elems);
  // One completion counter per point (fitset: per fit).
  L.counters = take(4 * (size_t)std::max(p->n_points, 1));
  L.queue = take(16);
  L.status = take(16);
  L.Rdense = take(p->kind == kChain ? scan_dense_bytes(p) : 0);
  L.tailpart = take(p->kind == kFitset ? 6 * 8 * p->total_slices : 0);
  L.fwd_order = take(4 * p->fwd_order.size());
  // Queued tail: one entry per tile and per fit.
  L.q_items = take(p->kind == kFitset ? 4 * ((size_t)p->tile_capacity + p->n_probs) : 0);
  L.total = off;
}

void delete_plan(PlanBuild& b) {
  delete b.p;
  b.p = nullptr;
}

int device_limits(gna_plan* p) {
  // Host-only sizing must not touch the device: defaults for gfx950.
  p->cu_count = 256;
  p->lds_limit = 64 * 1024;
  p->lds_device = 64 * 1024;
  std::snprintf(p->arch, sizeof(p->arch), "gfx950");
  return GNA_OK;
}

int prepare(PlanBuild& b, int kind, const gna_model* model, const gna_problem* problems,
            int32_t n_probs, int32_t n_points, int32_t prec, const gna_launch_opts* opts) {
  int rc = validate_model(model);
  if (rc) return rc;
  if (prec != GNA_FP64 && prec != GNA_MIXED) return fail(GNA_E_INVAL, "bad prec %d", prec);
  if (!problems) return fail(GNA_E_INVAL, "problems NULL");
  if (n_probs < 1 || n_probs > 65535)
    return fail(GNA_E_INVAL, "number of problems %d outside 1..65535", n_probs);
  if (n_points < 1 || n_points > (1 << 24))
    return fail(GNA_E_INVAL, "number of points %d outside 1..2^24", n_points);
  if (opts) {
    const int t = opts->threads;
    if (t != 0 && t != 64 && t != 128 && t != 256 && t != 512 && t != 1024)
      return fail(GNA_E_INVAL, "opts.threads = %d not in {64,128,256,512,1024}", t);
    const int g = opts->lanes_per_bin;
    if (g != 0 && (g < 1 || g > 64 || (g & (g - 1))))
      return fail(GNA_E_INVAL, "opts.lanes_per_bin = %d not a power of two <= 64", g);
    if (opts->chunks < 0 || opts->chunks > 1024)
      return fail(GNA_E_INVAL, "opts.chunks = %d outside 0..1024", opts->chunks);
    if (opts->persistent < 0 || opts->persistent > 1)
      return fail(GNA_E_INVAL, "opts.persistent = %d not 0/1", opts->persistent);
    if (opts->smear_mfma < -1 || opts->smear_mfma > 3)
      return fail(GNA_E_INVAL, "opts.smear_mfma = %d not in -1..3", opts->smear_mfma);
    if (opts->no_shared_phases < 0 || opts->no_shared_phases > 1)
      return fail(GNA_E_INVAL, "opts.no_shared_phases = %d not 0/1", opts->no_shared_phases);
    if (opts->split_tail < 0 || opts->split_tail > 3)
      return fail(GNA_E_INVAL, "opts.split_tail = %d not in 0..3", opts->split_tail);
    if (opts->split_tail == 3 && kind != kFitset)
      return fail(GNA_E_INVAL, "opts.split_tail = 3 needs a fitset plan");
  }
  for (int i = 0; i < n_probs; ++i) {
    rc = validate_problem(problems + i, i);
    if (rc) return rc;
  }
  gna_plan* p = new (std::nothrow) gna_plan();
  if (!p) return fail(GNA_E_INVAL, "out of host memory");
  b.p = p;
  p->kind = kind;
  p->prec = prec;
  p->n_probs = n_probs;
  p->n_points = n_points;
  p->model = *model;
  p->max_bins = 0;
  p->ws = nullptr;
  p->share_allowed = (opts && opts->no_shared_phases) ? 0 : 1;
  p->share_phases = p->share_allowed;
  device_limits(p);
  int64_t pts = 0, bins = 0, edges = 0, Ls = 0, slices = 0, band = 0;
  for (int i = 0; i < n_probs; ++i) {
    const gna_problem& q = problems[i];
    ProbDev pd{};
    pd.n_bins = q.n_bins;
    pd.order = q.gl_order;
    pd.n_sub = q.n_sub;
    pd.ppb = q.gl_order * q.n_sub;
    pd.n_L = q.n_L;
    pd.pt_off = pts;
    pd.bin_off = bins;
    pd.edge_off = edges;
    pd.L_off = Ls;
    pd.slice_off = slices;
    const size_t s0 = p->slices.size();
    const int64_t nband = build_slices(q.edges, q.n_bins, model->res_a, p->slices);
    for (size_t s = s0; s < p->slices.size(); ++s) {
      p->slices[s].off += band;
      b.slice_prob.push_back(i);
    }
    pd.n_slices = (int)(p->slices.size() - s0);
    band += nband;
    slices += pd.n_slices;
    pts += (int64_t)q.n_bins * pd.ppb;
    bins += q.n_bins;
    edges += q.n_bins + 1;
    Ls += q.n_L;
    p->max_bins = std::max(p->max_bins, q.n_bins);
    p->probs.push_back(pd);
    for (int j = 0; j <= q.n_bins; ++j) b.edges.push_back(q.edges[j]);
    for (int j = 0; j < q.n_bins; ++j) b.data.push_back(q.data[j]);
    for (int r = 0; r < q.n_L; ++r) {
      b.L.push_back(q.L_km[r]);
      b.wL.push_back(q.wL ? q.wL[r] : 1.0 / q.n_L);
    }
  }
  p->total_pts = pts;
  p->total_bins = bins;
  p->total_slices = slices;
  p->total_band = band;
  if (kind == kFitset) {
    // Tail work items in longest-first order (each slice's cost is its
    // number of diagonals), so the wide launch does not end on a few long
    // slices.
    const std::vector<SliceDev>& v = p->slices;
    std::vector<int32_t>& out = p->fwd_order;
    out.resize(v.size());
    for (size_t i = 0; i < v.size(); ++i) out[i] = (int32_t)i;
    std::stable_sort(out.begin(), out.end(),
                     [&](int32_t a, int32_t b) { return v[a].nd > v[b].nd; });
  }
  p->edges_host = b.edges;
  p->L_host = b.L;
  p->wL_host = b.wL;
  p->data_host = b.data;
  p->slice_prob_host = b.slice_prob;
  // Chunk cap, scratch and tile capacity for every shape the plan may run.
  if (opts && opts->chunks > 0)
    p->ccap = opts->chunks;
  else if (kind == kChain)
    p->ccap = std::max(1, std::min(64, (4096 + n_points - 1) / n_points));
  else
    p->ccap = 4;
  p->scratch_elems = 0;
  p->tile_capacity = 0;
  if (kind == kChain) {
    p->scratch_elems = (int64_t)n_points * p->ccap * 5 * p->probs[0].n_bins;
  } else {
    for (auto& pd : p->probs) {
      const int c = std::min(p->ccap, pd.ppb * pd.n_L);
      pd.scratch_off = p->scratch_elems;
      p->scratch_elems += (int64_t)c * 5 * pd.n_bins;
      p->tile_capacity += (int64_t)((pd.n_bins + 3) / 4) * c;
    }
  }
  // Shape: automatic, overridden field by field by opts.
  Shape sh = auto_shape(p);
  if (opts) {
    if (opts->threads) sh.threads = opts->threads;
    if (opts->lanes_per_bin) sh.G = std::min(opts->lanes_per_bin, sh.threads);
    if (opts->chunks) sh.C = opts->chunks;
    sh.persistent = opts->persistent;
    if (opts->smear_mfma >= 1) sh.mfma = opts->smear_mfma;
    if (opts->split_tail) sh.split = opts->split_tail - 1;  // 1, 2, 3 -> fused, split, queued
    p->tail_pin = opts->split_tail;
    if (sh.split == 2) sh.persistent = 1;
  }
  if (kind == kChain && (!opts || opts->smear_mfma == -1) && scan_supported(p) &&
      n_points >= 64)
    sh.mfma = 1;
  p->shape = sh;
  compute_layout(p, b);
  rc = apply_shape(p, sh, nullptr);  // validates; no workspace yet, nothing uploaded
  if (!rc && kind == kChain && !sh.mfma && !p->tail_pin && p->n_tiles > 1) {
    // Several tiles per point: by default the point pass and the per-point
    // tails go in two launches (the launch boundary orders the bin sums,
    // instead of a release and a completion count in every tile).
    sh.split = 1;
    rc = apply_shape(p, sh, nullptr);
  }
  if (rc) {
    delete_plan(b);
    return rc;
  }
  return GNA_OK;
}

int upload_and_build(PlanBuild& b, void* ws, size_t ws_bytes, hipStream_t s) {
  gna_plan* p = b.p;
  if (!ws) return fail(GNA_E_WORKSPACE, "workspace pointer is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(GNA_E_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < p->lay.total)
    return fail(GNA_E_WORKSPACE, "workspace has %zu bytes, plan needs %zu", ws_bytes,
                p->lay.total);
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  hipDeviceProp_t prop;
  rc = check_hip(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
  if (rc) return rc;
  p->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  p->lds_device = prop.sharedMemPerBlock > 0 ? (size_t)prop.sharedMemPerBlock : 64 * 1024;
  std::snprintf(p->arch, sizeof(p->arch), "%s", prop.gcnArchName);
  p->ws = (unsigned char*)ws;
  p->ws_bytes = ws_bytes;
  const Layout& L = p->lay;
  unsigned char* w = p->ws;
  auto up = [&](size_t off, const void* src, size_t bytes) {
    if (bytes == 0) return (int)GNA_OK;
    return check_hip(hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, s),
                     "hipMemcpyAsync (configuration upload)");
  };
  if ((rc = up(L.slices, p->slices.data(), sizeof(SliceDev) * p->slices.size()))) return rc;
  if ((rc = up(L.slice_prob, b.slice_prob.data(), 4 * b.slice_prob.size()))) return rc;
  if (p->kind == kFitset && (rc = up(L.fwd_order, p->fwd_order.data(), 4 * p->fwd_order.size())))
    return rc;
  if ((rc = up(L.L, b.L.data(), 8 * b.L.size()))) return rc;
  if ((rc = up(L.wL, b.wL.data(), 8 * b.wL.size()))) return rc;
  if ((rc = up(L.edges, b.edges.data(), 8 * b.edges.size()))) return rc;
  if ((rc = up(L.data, b.data.data(), 8 * b.data.size()))) return rc;
  // Problem descriptors and the tile list (and a sync for the host buffers).
  if ((rc = apply_shape(p, p->shape, s))) return rc;
  // Gauss-Legendre rules.
  double* glt = (double*)(w + L.gl);
  double* glw = glt + kGLTable;
  hipLaunchKernelGGL(gl_table_kernel, dim3(kMaxOrder), dim3(32), 0, s, glt, glw);
  if ((rc = check_hip(hipGetLastError(), "gl_table_kernel"))) return rc;
  // Quadrature energies and flux factors.
  int64_t max_pts = 0;
  for (auto& pd : p->probs) max_pts = std::max<int64_t>(max_pts, (int64_t)pd.n_bins * pd.ppb);
  const ProbDev* dprobs = (const ProbDev*)(w + L.probs);
  const dim3 qg((unsigned)((max_pts + 255) / 256), (unsigned)p->n_probs);
  if (p->prec == GNA_FP64)
    hipLaunchKernelGGL(quad_kernel<double>, qg, dim3(256), 0, s, dprobs,
                       (const double*)(w + L.edges), glt, glw, p->model, (double*)(w + L.E),
                       (double*)(w + L.f));
  else
    hipLaunchKernelGGL(quad_kernel<float>, qg, dim3(256), 0, s, dprobs,
                       (const double*)(w + L.edges), glt, glw, p->model, (double*)(w + L.E),
                       (float*)(w + L.f));
  if ((rc = check_hip(hipGetLastError(), "quad_kernel"))) return rc;
  // Banded smearing matrix.
  const SliceDev* dsl = (const SliceDev*)(w + L.slices);
  const int32_t* dsp = (const int32_t*)(w + L.slice_prob);
  if (p->prec == GNA_FP64)
    hipLaunchKernelGGL(band_kernel<double>, dim3((unsigned)p->total_slices), dim3(kSlice), 0, s,
                       dprobs, dsl, dsp, (const double*)(w + L.edges), p->model.res_a,
                       (double*)(w + L.Rv));
  else
    hipLaunchKernelGGL(band_kernel<float>, dim3((unsigned)p->total_slices), dim3(kSlice), 0, s,
                       dprobs, dsl, dsp, (const double*)(w + L.edges), p->model.res_a,
                       (float*)(w + L.Rv));
  if ((rc = check_hip(hipGetLastError(), "band_kernel"))) return rc;
  // Counters, queue and status start at zero (a fill kernel, not a memset).
  auto zero = [&](size_t off, int64_t n) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (uint32_t*)(w + off), n, 0u);
    return check_hip(hipGetLastError(), "fill_u32_kernel");
  };
  if ((rc = zero(L.counters, std::max(p->n_points, 1)))) return rc;
  if ((rc = zero(L.queue, 4))) return rc;
  if ((rc = zero(L.status, 4))) return rc;
  if (p->kind == kChain && scan_supported(p) && (rc = build_scan_tables(p, s))) return rc;
  return check_hip(hipStreamSynchronize(s), "hipStreamSynchronize (configuration)");
}

int create_common(int kind, const gna_model* model, const gna_problem* problems, int32_t n_probs,
                  int32_t n_points, int32_t prec, const gna_launch_opts* opts, void* ws,
                  size_t ws_bytes, void* stream, gna_plan** out) {
  clear_error();
  if (!out) return fail(GNA_E_INVAL, "out is NULL");
  *out = nullptr;
  PlanBuild b;
  int rc = prepare(b, kind, model, problems, n_probs, n_points, prec, opts);
  if (rc) return rc;
  rc = upload_and_build(b, ws, ws_bytes, (hipStream_t)stream);
  if (rc) {
    delete_plan(b);
    return rc;
  }
  *out = b.p;
  return GNA_OK;
}

int size_common(int kind, const gna_model* model, const gna_problem* problems, int32_t n_probs,
                int32_t n_points, int32_t prec, const gna_launch_opts* opts, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(GNA_E_INVAL, "bytes is NULL");
  PlanBuild b;
  int rc = prepare(b, kind, model, problems, n_probs, n_points, prec, opts);
  if (rc) return rc;
  *bytes = b.p->lay.total;
  delete_plan(b);
  return GNA_OK;
}

}  // namespace
}  // namespace gna

// ===========================================================================
// C ABI: lifecycle, status, tables.
// ===========================================================================
using namespace gna;

extern "C" int gna_chain_workspace_size(const gna_model* model, const gna_problem* problem,
                                        int32_t prec, int32_t max_batch,
                                        const gna_launch_opts* opts, size_t* bytes) {
  return size_common(kChain, model, problem, 1, max_batch, prec, opts, bytes);
}

extern "C" int gna_chain_create(const gna_model* model, const gna_problem* problem, int32_t prec,
                                int32_t max_batch, const gna_launch_opts* opts, void* ws_dev,
                                size_t ws_bytes, void* stream, gna_plan** out) {
  return create_common(kChain, model, problem, 1, max_batch, prec, opts, ws_dev, ws_bytes,
                       stream, out);
}

extern "C" int gna_fitset_workspace_size(const gna_model* model, const gna_problem* problems,
                                         int32_t n_fits, int32_t prec,
                                         const gna_launch_opts* opts, size_t* bytes) {
  if (n_fits < 1) return fail(GNA_E_INVAL, "n_fits = %d < 1", n_fits);
  return size_common(kFitset, model, problems, n_fits, n_fits, prec, opts, bytes);
}

extern "C" int gna_fitset_create(const gna_model* model, const gna_problem* problems,
                                 int32_t n_fits, int32_t prec, const gna_launch_opts* opts,
                                 void* ws_dev, size_t ws_bytes, void* stream, gna_plan** out) {
  if (n_fits < 1) return fail(GNA_E_INVAL, "n_fits = %d < 1", n_fits);
  return create_common(kFitset, model, problems, n_fits, n_fits, prec, opts, ws_dev, ws_bytes,
                       stream, out);
}

extern "C" int gna_chain_eval(gna_plan* plan, const double* params_dev, int32_t B,
                              double* chi2_dev, double* grad_dev, double* pred_dev,
                              void* stream) {
  clear_error();
  if (!plan || plan->kind != kChain) return fail(GNA_E_INVAL, "not a chain plan");
  if (B < 1 || B > plan->n_points)
    return fail(GNA_E_INVAL, "B = %d outside 1..max_batch = %d", B, plan->n_points);
  if (!params_dev || !chi2_dev) return fail(GNA_E_INVAL, "params or chi2 pointer is NULL");
  if (((uintptr_t)params_dev | (uintptr_t)chi2_dev | (uintptr_t)grad_dev | (uintptr_t)pred_dev) & 7)
    return fail(GNA_E_INVAL, "device pointers must be 8-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  if (plan->shape.mfma) return launch_scan(plan, params_dev, B, chi2_dev, grad_dev, pred_dev, s);
  return launch_chain(plan, params_dev, B, chi2_dev, grad_dev, pred_dev, s);
}

extern "C" int gna_fitset_eval(gna_plan* plan, const double* params_dev, double* chi2_dev,
                               double* grad_dev, double* pred_dev, void* stream) {
  clear_error();
  if (!plan || plan->kind != kFitset) return fail(GNA_E_INVAL, "not a fitset plan");
  if (!params_dev || !chi2_dev) return fail(GNA_E_INVAL, "params or chi2 pointer is NULL");
  if (((uintptr_t)params_dev | (uintptr_t)chi2_dev | (uintptr_t)grad_dev | (uintptr_t)pred_dev) & 7)
    return fail(GNA_E_INVAL, "device pointers must be 8-byte aligned");
  return launch_chain(plan, params_dev, plan->n_points, chi2_dev, grad_dev, pred_dev,
                      (hipStream_t)stream);
}

extern "C" int gna_plan_rebuild(gna_plan* plan, void* stream) {
  clear_error();
  if (!plan || !plan->ws) return fail(GNA_E_INVAL, "gna_plan_rebuild: plan is NULL");
  PlanBuild b;
  b.p = plan;
  b.L = plan->L_host;
  b.wL = plan->wL_host;
  b.edges = plan->edges_host;
  b.data = plan->data_host;
  b.slice_prob = plan->slice_prob_host;
  const int rc = upload_and_build(b, plan->ws, plan->ws_bytes, (hipStream_t)stream);
  b.p = nullptr;  // the caller keeps the plan
  return rc;
}

extern "C" int gna_plan_status(gna_plan* plan, void* stream, int32_t* device_status) {
  clear_error();
  if (!plan || !plan->ws) return fail(GNA_E_INVAL, "plan is NULL");
  hipStream_t s = (hipStream_t)stream;
  int rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize (status)");
  if (rc) return rc;
  uint32_t word = 0;
  rc = check_hip(hipMemcpy(&word, plan->ws + plan->lay.status, 4, hipMemcpyDeviceToHost),
                 "hipMemcpy (status word)");
  if (rc) return rc;
  if (device_status) *device_status = (int32_t)word;
  if (word) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s,
                       (uint32_t*)(plan->ws + plan->lay.status), (int64_t)4, 0u);
    rc = check_hip(hipStreamSynchronize(s), "clearing the status word");
    if (rc) return rc;
    if (word & kSpinTimeout)
      return fail(GNA_E_HIP, "device status word 0x%x: a queued tail gave up waiting for its "
                  "fit's point tiles (results invalid; rebuild the plan)", word);
    return fail(GNA_E_DOMAIN, "device status word 0x%x (%s%s)", word,
                (word & kBadMixing) ? "mixing parameter outside [0,1] " : "",
                (word & kBadPrediction) ? "prediction <= 0 or not finite" : "");
  }
  return GNA_OK;
}

extern "C" int gna_plan_shape(const gna_plan* plan, int32_t shape_out[7], int64_t* n_tiles) {
  clear_error();
  if (!plan) return fail(GNA_E_INVAL, "plan is NULL");
  // The MFMA scan kernel has its own tiling: 16 parameter points per tile,
  // one work-group of scan_threads lanes each (lanes per bin and chunks do
  // not apply).
  const bool mfma = plan->shape.mfma != 0;
  if (shape_out) {
    shape_out[0] = mfma ? scan_threads(plan) : plan->shape.threads;
    shape_out[1] = mfma ? 1 : plan->shape.G;
    shape_out[2] = mfma ? 1 : plan->shape.C;
    shape_out[3] = plan->shape.persistent;
    shape_out[4] = plan->shape.mfma;
    shape_out[5] = plan->share_phases;
    shape_out[6] = plan->shape.split;
  }
  if (n_tiles) *n_tiles = mfma ? (int64_t)(plan->n_points + 15) / 16 : plan->n_tiles;
  return GNA_OK;
}

extern "C" int gna_plan_destroy(gna_plan* plan) {
  delete plan;
  return GNA_OK;
}

extern "C" int gna_gl_nodes_dev(int32_t order, double* t_dev, double* w_dev, void* stream) {
  clear_error();
  if (order < 1 || order > kMaxOrder)
    return fail(GNA_E_INVAL, "order = %d outside 1..%d", order, kMaxOrder);
  if (!t_dev || !w_dev) return fail(GNA_E_INVAL, "NULL output");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(gl_one_kernel, dim3(1), dim3(32), 0, s, order, t_dev, w_dev);
  int rc = check_hip(hipGetLastError(), "gl_one_kernel");
  if (rc) return rc;
  return check_hip(hipStreamSynchronize(s), "hipStreamSynchronize (gl nodes)");
}

namespace {
std::mutex g_gl_stage_mu;  // one host-output rule at a time (shared staging array)
}

extern "C" int gna_gl_nodes(int32_t order, double* t_host, double* w_host) {
  clear_error();
  if (order < 1 || order > kMaxOrder)
    return fail(GNA_E_INVAL, "order = %d outside 1..%d", order, kMaxOrder);
  if (!t_host || !w_host) return fail(GNA_E_INVAL, "NULL output");
  std::lock_guard<std::mutex> lock(g_gl_stage_mu);
  hipLaunchKernelGGL(gl_stage_kernel, dim3(1), dim3(32), 0, nullptr, (int)order);
  int rc = check_hip(hipGetLastError(), "gl_stage_kernel");
  if (rc) return rc;
  // Copies on the null stream run after the kernel and return when done.
  if ((rc = check_hip(hipMemcpyFromSymbol(t_host, HIP_SYMBOL(gl_stage), sizeof(double) * order, 0,
                                          hipMemcpyDeviceToHost),
                      "hipMemcpyFromSymbol (nodes)")))
    return rc;
  return check_hip(hipMemcpyFromSymbol(w_host, HIP_SYMBOL(gl_stage), sizeof(double) * order,
                                       sizeof(double) * kMaxOrder, hipMemcpyDeviceToHost),
                   "hipMemcpyFromSymbol (weights)");
}

extern "C" int gna_plan_tables(const gna_plan* plan, int32_t index, double* E_dev, double* f_dev,
                               double* R_dev, void* stream) {
  clear_error();
  if (!plan || !plan->ws) return fail(GNA_E_INVAL, "plan is NULL");
  if (index < 0 || index >= plan->n_probs)
    return fail(GNA_E_INVAL, "problem index %d outside 0..%d", index, plan->n_probs - 1);
  hipStream_t s = (hipStream_t)stream;
  const ProbDev& pd = plan->probs[index];
  const int64_t npts = (int64_t)pd.n_bins * pd.ppb;
  const unsigned char* w = plan->ws;
  int rc;
  if (E_dev) {
    rc = check_hip(hipMemcpyAsync(E_dev, w + plan->lay.E + 8 * pd.pt_off, 8 * npts,
                                  hipMemcpyDeviceToDevice, s),
                   "hipMemcpyAsync (E table)");
    if (rc) return rc;
  }
  if (f_dev) {
    const unsigned g = (unsigned)((npts + 255) / 256);
    if (plan->prec == GNA_FP64)
      hipLaunchKernelGGL(widen_kernel<double>, dim3(g), dim3(256), 0, s,
                         (const double*)(w + plan->lay.f) + pd.pt_off, npts, f_dev);
    else
      hipLaunchKernelGGL(widen_kernel<float>, dim3(g), dim3(256), 0, s,
                         (const float*)(w + plan->lay.f) + pd.pt_off, npts, f_dev);
    if ((rc = check_hip(hipGetLastError(), "widen_kernel"))) return rc;
  }
  if (R_dev) {
    const int64_t n2 = (int64_t)pd.n_bins * pd.n_bins;
    const unsigned g = (unsigned)((n2 + 255) / 256);
    const ProbDev* dp = (const ProbDev*)(w + plan->lay.probs);
    const SliceDev* ds = (const SliceDev*)(w + plan->lay.slices);
    if (plan->prec == GNA_FP64)
      hipLaunchKernelGGL(dense_kernel<double>, dim3(g), dim3(256), 0, s, dp, index, ds,
                         (const double*)(w + plan->lay.Rv), R_dev);
    else
      hipLaunchKernelGGL(dense_kernel<float>, dim3(g), dim3(256), 0, s, dp, index, ds,
                         (const float*)(w + plan->lay.Rv), R_dev);
    if ((rc = check_hip(hipGetLastError(), "dense_kernel"))) return rc;
  }
  return GNA_OK;
}
