// The fused prediction chain on the GPU: one kernel evaluates, for a set of
// parameter points, every step from the oscillation probability to chi^2 and
// its gradient.
//
// Work decomposition.  A tile is (parameter point, block of bins, chunk of
// each bin's quadrature points).  Inside a tile, G lanes share a bin: each
// lane walks the bin's points (all baselines, Fig. 4), or, when a bin has
// fewer than two points per lane, its (point, baseline) items, and
// accumulates
//   mu0_j = sum_k f_k Pbar_k   and   J0_jc = sum_k f_k d Pbar_k / d theta_c,
// then the G lanes are summed with cross-lane shuffles.  When a point's bins
// fit one tile the results stay in LDS; otherwise each tile writes its
// partial sums to the scratch region and the last tile of the point (agent-
// scope counter, release/acquire fences) adds the chunks in a fixed order and
// runs the tail.  Results are therefore independent of scheduling.  An
// uneven batch can instead split the tail off into wide launches over all
// fits (tail_fwd / tail_final below).
//
// Tail (one work-group per point), one pass over the banded R with the
// tangent columns carried along (one wavefront per 64-row slice):
//   s_i     = sum_j R_ij mu0_j,  t_ic = sum_j R_ij J0_jc
//   nu_i    = norm s_i                                      (FP64)
//   chi2    = 2 sum_i [nu_i - d_i + d_i ln(d_i / nu_i)]     (FP64)
//   gnu_i   = 2 (1 - d_i / nu_i)                            (FP64)
//   grad_c  = norm sum_i gnu_i t_ic,  grad_norm = sum_i gnu_i s_i      (FP64 sums)
// which equals the adjoint form norm sum_j gmu_j J0_jc with gmu = R^T gnu,
// without a second pass over R.
#include <cmath>

#include "gna_internal.h"
#include "gna_math.h"
#include "lanes.h"

namespace gna {
namespace {

template <class R>
__device__ __forceinline__ R rfma(R a, R b, R c);
template <>
__device__ __forceinline__ double rfma<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float rfma<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// Band loads issued back to back in the smearing loops (32 VGPRs of
// operands either way; 16 FP64 loads measured no faster).
template <class R>
constexpr int kTailBatch = sizeof(R) == 8 ? 8 : 16;

// Dynamic LDS of one work-group (sizes in chain_lds):
//   vec   [5][vs]             mu0 and the four J0 columns of the point
//                             (vs = 0: they stay in the scratch region)
//   part  [5][threads]        partial smearing sums of the diagonal chunks
//                             (absent when kf_cap == 1)
//   red   [waves][6]          per-wave chi2 and gradient partials
//   flag
struct TileLds {
  unsigned char* base;
  int threads;
  int vs;
  int kf_cap;
  __device__ static size_t align16(size_t x) { return (x + 15) & ~size_t(15); }
  template <class R>
  __device__ size_t o_part() const { return align16((size_t)5 * vs * sizeof(R)); }
  template <class R>
  __device__ size_t o_red() const {
    return o_part<R>() + (kf_cap > 1 ? align16((size_t)5 * threads * sizeof(R)) : 0);
  }
  template <class R>
  __device__ R* vec() const { return reinterpret_cast<R*>(base); }
  template <class R>
  __device__ R* part() const { return reinterpret_cast<R*>(base + o_part<R>()); }
  template <class R>
  __device__ double* red() const { return reinterpret_cast<double*>(base + o_red<R>()); }
  template <class R>
  __device__ int* flag() const { return reinterpret_cast<int*>(red<R>() + (threads / kWave) * 6); }
};

// acc[k] = sum_{d0 <= d < d1} R_{i, i+dlo+d} V[k vst + i + dlo + d], k < NC, for
// row i = 64 s + lane of one slice of the band (diagonal layout: entry (l, d)
// at off + (d - dlo) * 64 + l), summed over d in ascending order.  The band
// stores exact zeros at columns outside [0, nb), which read V at column 0
// instead (finite), so they add 0.  The band loads of a batch go out together, the
// vector reads follow them; the last, partial batch is issued the same way
// (its missing diagonals load nothing and add exact zeros), so a wavefront
// waits for memory once per batch, not once per diagonal.
template <class R>
constexpr int kDotBatch = sizeof(R) == 8 ? 8 : 16;
template <class R, int NC>
__device__ __forceinline__ void slice_dot(const R* __restrict__ Rv, const SliceDev& sd, int s,
                                          int lane, int nb, const R* __restrict__ V, int vst,
                                          int d0, int d1, R (&acc)[NC]) {
  const R* rv = Rv + sd.off + lane;
  const int jb = s * kSlice + lane + sd.dlo;  // column of diagonal 0
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = R(0);
  for (int dd = d0; dd < d1; dd += kDotBatch<R>) {
    R x[kDotBatch<R>];
#pragma unroll
    for (int u = 0; u < kDotBatch<R>; ++u)
      x[u] = (dd + u < d1) ? rv[(int64_t)(dd + u) * kSlice] : R(0);
    __builtin_amdgcn_sched_barrier(0);
    // The vector entries of four diagonals are read together, then used:
    // otherwise each read waits before its FMA.
#pragma unroll
    for (int u0 = 0; u0 < kDotBatch<R>; u0 += 4) {
      R y[4][NC];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int jj = jb + dd + u0 + u;
        const int jc = (unsigned)jj < (unsigned)nb ? jj : 0;
#pragma unroll
        for (int k = 0; k < NC; ++k) y[u][k] = V[k * vst + jc];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] = rfma<R>(x[u0 + u], y[u][k], acc[k]);
    }
  }
}

// sum over chunks c < C of sc[(c*5 + comp)*nb + j], added in the order
// c = 0, 1, ...: the loads of eight chunks are issued before any is added
// (the partials come from other work-groups, so each load is a trip to
// memory); missing chunks of the last eight add exact zeros.
template <class R>
__device__ __forceinline__ R sum_chunks(const R* sc, int C, int comp, int nb, int j) {
  R s = R(0);
  for (int c = 0; c < C; c += 8) {
    R v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = (c + u < C) ? sc[(int64_t)((c + u) * 5 + comp) * nb + j] : R(0);
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  return s;
}

// vl[c vs + jj] = the chunk sum (as sum_chunks) of entry e = c nb + jj, for
// this thread's entries e = tid, tid + NT, ... < n: U entries at a time, all
// their chunk loads in flight together.
template <class R, int U>
__device__ __forceinline__ void chunk_sums_to_lds(const R* sc, int C, int nb, int n, R* vl, int vs,
                                                  int tid, int NT) {
  for (int e0 = tid; e0 < n; e0 += U * NT) {
    R sum[U];
    int cc[U], jj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = min(e0 + u * NT, n - 1);
      cc[u] = e / nb;
      jj[u] = e - cc[u] * nb;
      sum[u] = R(0);
    }
    for (int c = 0; c < C; c += 8) {
      R v[U][8];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < 8; ++k)
          v[u][k] = (e0 + u * NT < n && c + k < C)
                        ? sc[(int64_t)((c + k) * 5 + cc[u]) * nb + jj[u]] : R(0);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < 8; ++k) sum[u] += v[u][k];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + u * NT < n) vl[cc[u] * vs + jj[u]] = sum[u];
  }
}

// Baseline constants of the current tile's problem, staged once per tile so
// the per-baseline loop reads LDS (a broadcast) instead of waiting on memory.
struct BaseLds {
  double kl[kMaxBaselines];  // K L_r
  double w[kMaxBaselines];   // w_r
};

// The tail of one point (a fit, for a fitset) once its bin sums are
// complete: the chunk sums (unless the point was one tile whose sums are
// already in LDS), nu = norm R mu0 with the four tangent columns through R,
// the chi^2 terms, the gradient, in one work-group.  vl / sc: the point's
// vectors in LDS (L.vs > 0) or in chunk 0 of its scratch region.
template <class R, bool GRAD, int UNROLL = 2, class BadF>
__device__ void point_tail(const ChainArgs<R>& a, const ProbDev& pd, int point, const double* th,
                           BadF bad_of, const TileLds& L, bool single) {
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const int nb = pd.n_bins;
  const bool vlds = L.vs > 0;
  R* vl = L.vec<R>();
  R* sc = a.scratch + (a.tiles ? pd.scratch_off : (int64_t)point * a.scratch_stride);
  // ---- tail ----------------------------------------------------------------
  constexpr int NC = GRAD ? 5 : 1;
  const int C = pd.C;
  const double* dat = a.data + pd.bin_off;
  // (wave is uniform over the wavefront: its descriptor reads are scalar.)
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int lane = tid - (tid / kWave) * kWave;
  const int nwaves = NT / kWave;
  const int ns = pd.n_slices;
  const SliceDev* slices = a.slices + pd.slice_off;
  // Smearing work items (slice, chunk of its diagonals) over all waves; the
  // descriptor of this wavefront's first item is requested now.
  const int Kf = min(L.kf_cap, max(1, nwaves / ns));
  const SliceDev sd_first = slices[min(wave, ns * Kf - 1) / Kf];
  // This thread's first row of the chi^2 pass below when the slices are
  // split into chunks (row tid); requested now so that its latency overlaps.
  const double d_first = (tid < nb) ? dat[tid] : 0.0;
  // Entries e = c nb + jj of the NC vectors, UNROLL per trip so that their
  // chunk loads are in flight together (the in-place form: two).
  if (vlds) {
    if (!single) chunk_sums_to_lds<R, UNROLL>(sc, C, nb, NC * nb, vl, L.vs, tid, NT);
  } else if (C > 1) {
    // In place into chunk 0: each entry is read and written by one thread.
#pragma unroll 2
    for (int e = tid; e < NC * nb; e += NT) {
      const int c = e / nb, jj = e - (e / nb) * nb;
      const R v = sum_chunks<R>(sc, C, c, nb, jj);
      sc[c * nb + jj] = v;
    }
  }
  __syncthreads();

  const double norm = th[4];
  double* pred = a.pred ? (a.tiles ? a.pred + pd.bin_off : a.pred + (int64_t)point * nb)
                        : nullptr;
  double chi = 0.0;
  double gs[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  bool badnu = false;
  // Row i (data d) from s_i = acc[0] and t_ic = acc[1 + c].
  auto finish = [&](int i, double d, const R(&acc)[NC]) {
    const double nu = norm * (double)acc[0];
    if (!(nu > 0.0) || !isfinite(nu)) badnu = true;
    const double ratio = quot_pos(d, nu);
    chi += dfma(d, log_pos(d > 0.0 ? ratio : 1.0), nu - d);  // d = 0 takes ln 1 = 0
    if (GRAD) {
      const double gn = 2.0 * (1.0 - ratio);
#pragma unroll
      for (int c = 0; c < 4; ++c) gs[c] = dfma(gn, (double)acc[(1 + c) % NC], gs[c]);
      gs[4] = dfma(gn, (double)acc[0], gs[4]);
    }
    if (pred) pred[i] = nu;
  };

  // Smearing: each wavefront's items; with one chunk per slice each
  // wavefront finishes its own rows.
  const int PS = ns * kSlice;
  R* part = L.part<R>();  // [Kf][NC][PS]: Kf * PS <= threads
  auto run_item = [&](int item, const SliceDev& sd) {
    const int s = item / Kf, kap = item - (item / Kf) * Kf;
    const int csz = (sd.nd + Kf - 1) / Kf;
    const int d0 = min(sd.nd, kap * csz), d1 = min(sd.nd, d0 + csz);
    const int i = s * kSlice + lane;
    const double di = (Kf == 1 && i < nb) ? dat[i] : 0.0;
    R acc[NC];
    if (vlds)
      slice_dot<R, NC>(a.Rv, sd, s, lane, nb, vl, L.vs, d0, d1, acc);
    else
      slice_dot<R, NC>(a.Rv, sd, s, lane, nb, sc, nb, d0, d1, acc);
    if (i < nb) {
      if (Kf == 1) {
        finish(i, di, acc);
      } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) part[(kap * NC + c) * PS + i] = acc[c];
      }
    }
  };
  if (wave < ns * Kf) run_item(wave, sd_first);
  for (int item = wave + nwaves; item < ns * Kf; item += nwaves) run_item(item, slices[item / Kf]);
  if (Kf > 1) {
    __syncthreads();
    for (int i = tid; i < nb; i += NT) {
      R acc[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = part[c * PS + i];
      for (int kap = 1; kap < Kf; ++kap) {
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += part[(kap * NC + c) * PS + i];
      }
      finish(i, i == tid ? d_first : dat[i], acc);
    }
  }
  if (badnu) __hip_atomic_fetch_or(a.status, (uint32_t)kBadPrediction, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
  double* red = L.red<R>();
  chi = wave_total(chi);
  if (GRAD) {
#pragma unroll
    for (int c = 0; c < 5; ++c) gs[c] = wave_total(gs[c]);
  }
  if (lane == kWave - 1) {
    red[wave * 6] = chi;
    if (GRAD) {
#pragma unroll
      for (int c = 0; c < 5; ++c) red[wave * 6 + 1 + c] = gs[c];
    }
  }
  __syncthreads();
  if (tid == 0) {
    double chisum = 0.0, g5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < nwaves; ++w) {
      chisum += red[w * 6];
      if (GRAD) {
#pragma unroll
        for (int c = 0; c < 5; ++c) g5[c] += red[w * 6 + 1 + c];
      }
    }
    const bool bad = bad_of();  // (after the sums: the parameters' loads are long done)
    if (bad) __hip_atomic_fetch_or(a.status, (uint32_t)kBadMixing, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    a.chi2[point] = bad ? NAN : 2.0 * chisum;
    if (GRAD && a.grad) {
      double* gp = a.grad + 5 * (int64_t)point;
#pragma unroll
      for (int c = 0; c < 4; ++c) gp[c] = bad ? NAN : norm * g5[c];
      gp[4] = bad ? NAN : g5[4];
    }
  }
}

template <class R, bool GRAD, bool SPLIT, bool QUEUED = false>
__device__ void process_tile(const ChainArgs<R>& a, int64_t t, const TileLds& L, BaseLds& bl) {
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  TileDev td;
  if (a.tiles) {
    td = a.tiles[t];
  } else {
    const ProbDev& p0 = a.probs[0];
    td.point = (int32_t)(t / a.tiles_per_point);
    const int local = (int)(t - (int64_t)td.point * a.tiles_per_point);
    td.prob = 0;
    td.bb = local / p0.C;
    td.chunk = local - td.bb * p0.C;
  }
  const ProbDev pd = a.probs[td.prob];
  // The point's parameters (uniform over the work-group): from the device
  // array, or passed by value for a single point.
  double thv[5];
  if (a.params) {
#pragma unroll
    for (int c = 0; c < 5; ++c) thv[c] = a.params[5 * (int64_t)td.point + c];
  } else {
#pragma unroll
    for (int c = 0; c < 5; ++c) thv[c] = a.pin[c];
  }
  const double* th = thv;
  for (int r = tid; r < pd.n_L; r += NT) {
    bl.kl[r] = kPhase * a.L[pd.L_off + r];
    bl.w[r] = a.wL[pd.L_off + r];
  }
  const PeeCoef<R> k = pee_coef<R>(th);
  __syncthreads();

  // ---- point pass --------------------------------------------------------
  const int G = pd.G;
  const int lb = tid / G, g = tid - (tid / G) * G;
  const int j = td.bb * pd.bins_per_tile + lb;
  // Chunk td.chunk of the bin's units: points, or (point, baseline) items
  // it = kk n_L + r when the plan splits items.
  const int units = pd.by_item ? pd.ppb * pd.n_L : pd.ppb;
  const int k0 = (int)((int64_t)td.chunk * units / pd.C);
  const int k1 = (int)((int64_t)(td.chunk + 1) * units / pd.C);
  R mu = R(0);
  R J[4] = {R(0), R(0), R(0), R(0)};
  if (lb < pd.bins_per_tile && j < pd.n_bins && pd.by_item) {
    // One evaluation per trip: lane g takes items k0 + g, k0 + g + G, ...;
    // (kk, r) step by G = gq n_L + gr without a division per item.
    const int64_t base = pd.pt_off + (int64_t)j * pd.ppb;
    const int nL = pd.n_L;
    const int gq = G / nL, gr = G - (G / nL) * nL;
    int it = k0 + g;
    int kk = it / nL, r = it - (it / nL) * nL;
    for (; it < k1; it += G) {
      const double E = a.E[base + kk];
      const R fk = a.f[base + kk];
      const double q = phase_per_ev2(bl.kl[r], E);
      const R fw = fk * (R)bl.w[r];
      R P, dP[4];
      pee_point<R, GRAD>(k, q, P, dP);
      mu = rfma<R>(fw, P, mu);
      if (GRAD) {
#pragma unroll
        for (int c = 0; c < 4; ++c) J[c] = rfma<R>(fw, dP[c], J[c]);
      }
      kk += gq;
      r += gr;
      if (r >= nL) {
        r -= nL;
        ++kk;
      }
    }
  } else if (lb < pd.bins_per_tile && j < pd.n_bins) {
    const int64_t base = pd.pt_off + (int64_t)j * pd.ppb;
    const int nL = pd.n_L;
    // Software-pipelined: the next point's E and f and the next baseline's
    // constants are requested before the current evaluation.
    int kk = k0 + g;
    double En = (kk < k1) ? a.E[base + kk] : 1.0;
    R fn = (kk < k1) ? a.f[base + kk] : R(0);
    for (; kk < k1; kk += G) {
      const double E = En;
      const R fk = fn;
      if (kk + G < k1) {
        En = a.E[base + kk + G];
        fn = a.f[base + kk + G];
      }
      R pb = R(0);
      R dpb[4] = {R(0), R(0), R(0), R(0)};
      double kln = bl.kl[0], wn = bl.w[0];
      for (int r = 0; r < nL; ++r) {
        const double klr = kln, wrd = wn;
        const int rn = (r + 1 < nL) ? r + 1 : r;
        kln = bl.kl[rn];
        wn = bl.w[rn];
        __builtin_amdgcn_sched_barrier(0);  // keep the request ahead of the math
        const double q = phase_per_ev2(klr, E);
        const R wr = (R)wrd;
        R P, dP[4];
        pee_point<R, GRAD>(k, q, P, dP);
        pb = rfma<R>(wr, P, pb);
        if (GRAD) {
#pragma unroll
          for (int c = 0; c < 4; ++c) dpb[c] = rfma<R>(wr, dP[c], dpb[c]);
        }
      }
      mu = rfma<R>(fk, pb, mu);
      if (GRAD) {
#pragma unroll
        for (int c = 0; c < 4; ++c) J[c] = rfma<R>(fk, dpb[c], J[c]);
      }
    }
  }
  // Sum the G lanes of each bin (groups are aligned inside a wavefront).
  if (GRAD) {
    R v[5] = {mu, J[0], J[1], J[2], J[3]};
    group_sums(v, G);
    mu = v[0];
#pragma unroll
    for (int c = 0; c < 4; ++c) J[c] = v[1 + c];
  } else {
    R v[1] = {mu};
    group_sums(v, G);
    mu = v[0];
  }

  const int nb = pd.n_bins;
  if (SPLIT) {
    // Split tail: every tile leaves its partial sums in the scratch region;
    // the tail kernels (a fitset's, or a chain plan's per-point tail) read
    // them after this launch.  Queued tail: the tile
    // then counts itself done for its fit, releasing its sums at agent scope
    // (every wavefront's stores acknowledged first, one L2 write-back by the
    // release-ordered increment), for the tail items of the same launch.
    R* sc = a.scratch + (a.tiles ? pd.scratch_off : (int64_t)td.point * a.scratch_stride);
    if (g == 0 && lb < pd.bins_per_tile && j < nb) {
      sc[(int64_t)(td.chunk * 5) * nb + j] = mu;
      if (GRAD) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sc[(int64_t)(td.chunk * 5 + 1 + c) * nb + j] = J[c];
      }
    }
    if (QUEUED) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      if (tid == 0)
        __hip_atomic_fetch_add(&a.counters[td.point], 1u, __ATOMIC_ACQ_REL,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  const int tiles_of_point = pd.n_bin_blocks * pd.C;
  const bool single = (tiles_of_point == 1);
  // The point's vectors: in LDS (component k of bin jj at vl[k vs + jj]) when
  // they fit, else in chunk 0 of the scratch region (sc[k nb + jj]).
  const bool vlds = L.vs > 0;
  R* vl = L.vec<R>();
  R* sc = a.scratch + (a.tiles ? pd.scratch_off : (int64_t)td.point * a.scratch_stride);
  if (g == 0 && lb < pd.bins_per_tile && j < nb) {
    if (single && vlds) {
      vl[j] = mu;
      if (GRAD) {
#pragma unroll
        for (int c = 0; c < 4; ++c) vl[(1 + c) * L.vs + j] = J[c];
      }
    } else {
      sc[(int64_t)(td.chunk * 5) * nb + j] = mu;
      if (GRAD) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sc[(int64_t)(td.chunk * 5 + 1 + c) * nb + j] = J[c];
      }
    }
  }
  int* flag = L.flag<R>();
  if (!single) {
    // Release this tile's partial sums at agent scope with one L2 write-back
    // per tile instead of one per wavefront: each wavefront first waits
    // until its own stores are acknowledged by the L2 (the barrier alone does
    // not wait for them), then thread 0's release-acquire increment writes
    // the L2 back before it counts the tile.
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (tid == 0) {
      const uint32_t prev = __hip_atomic_fetch_add(&a.counters[td.point], 1u, __ATOMIC_ACQ_REL,
                                                   __HIP_MEMORY_SCOPE_AGENT);
      *flag = (prev + 1 == (uint32_t)tiles_of_point) ? 1 : 0;
    }
    __syncthreads();
    if (*flag == 0) return;  // not the last tile of this point
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the other tiles' partial sums
    if (tid == 0) a.counters[td.point] = 0u;  // ready for the next evaluation
  } else {
    __syncthreads();
  }

  point_tail<R, GRAD>(a, pd, td.point, th, [&] { return k.bad; }, L, single);
}

template <class R, bool GRAD, bool PERSIST, bool SPLIT>
__global__ void __launch_bounds__(1024) chain_kernel(ChainArgs<R> a, int vs, int kf_cap) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  TileLds L{lds_raw, (int)blockDim.x, vs, kf_cap};
  __shared__ BaseLds bl;
  if (!PERSIST) {
    process_tile<R, GRAD, SPLIT>(a, (int64_t)blockIdx.x, L, bl);
    return;
  }
  __shared__ uint32_t next;
  for (;;) {
    if (threadIdx.x == 0)
      next = __hip_atomic_fetch_add(&a.queue[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t t = next;
    __syncthreads();
    if (t >= a.n_tiles) break;
    process_tile<R, GRAD, SPLIT>(a, t, L, bl);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // Every group increments the exit count once, after its last queue
    // fetch; the last one resets the queue for the next launch.
    const uint32_t done = __hip_atomic_fetch_add(&a.queue[1], 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (done + 1 == gridDim.x) {
      a.queue[0] = 0u;
      a.queue[1] = 0u;
    }
  }
}

// Two-launch form of a chain plan (split tail): after the point pass of all
// tiles, one work-group per parameter point sums the point's chunks and runs
// its tail.  The launch boundary orders the sums; there is no completion
// counter and no cross-work-group release, which a one-launch hand-off pays
// in every tile (an L2 write-back, then an atomic round trip).  The tail has
// its own width, kChainTailThreads lanes whatever the point pass used (its
// diagonal chunks per slice follow the width, so the last bits match the
// one-launch form of a shape of that width).
template <class R, bool GRAD>
__global__ void __launch_bounds__(kChainTailThreads) chain_tail_kernel(ChainArgs<R> a, int vs,
                                                                      int kf_cap) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  TileLds L{lds_raw, (int)blockDim.x, vs, kf_cap};
  const int point = blockIdx.x;
  double th[5];
  if (a.params) {
#pragma unroll
    for (int c = 0; c < 5; ++c) th[c] = a.params[5 * (int64_t)point + c];
  } else {
#pragma unroll
    for (int c = 0; c < 5; ++c) th[c] = a.pin[c];
  }
  // The chunk sums go out before anything waits for the parameters: P_ee's
  // mixing check is taken at the end, norm when the first row finishes.
  point_tail<R, GRAD, 4>(a, a.probs[0], point, th, [&] { return pee_coef<R>(th).bad; }, L,
                         false);
}

// ---- split tail (uneven batches) ------------------------------------------
// With a split tail the point pass above only writes every fit's bin sums;
// two more launches finish the chain with the whole GPU on each step:
//   tail_fwd    one wavefront per 64-row slice of any fit: nu_i = norm (R mu0)_i,
//               the chi^2 terms, gnu_i = 2 (1 - d_i / nu_i) and, with the
//               gradient, the tangent rows (R J0)_ic, all from one pass over
//               the slice's diagonals; the slice's partials are
//               sum_i chi2 terms, sum_i gnu_i (R J0)_ic and sum_i gnu_i (R mu0)_i
//   tail_final  per fit: the slice partials added in a fixed order
// Carrying the four tangent columns through the smearing replaces the
// adjoint pass over R^T: sum_j gmu_j J0_jc = sum_i gnu_i (R J0)_ic, so the
// band is read once per evaluation instead of twice.
template <class R>
struct TailArgs {
  const ProbDev* probs;
  const SliceDev* slices;
  const int32_t* slice_prob;  // fit of each slice
  const int32_t* order;       // the launch's slices, longest first
  int64_t n_items;            // slices of all fits
  int32_t n_fits;
  const R* Rv;
  const double* data;
  const double* params;
  const R* scratch;
  double* part;               // [n_items][6]  chi2 partial, 5 gradient partials
  double* pred;
  uint32_t* status;
  double* chi2;
  double* grad;
};

constexpr int kTailWaves = 4;  // wavefronts (slices) per work-group

// Diagonals per staged window.  A gradient window holds five vectors
// (mu0 and the four tangents), so FP64 halves it to keep a work-group's LDS
// (and with it the number of resident work-groups) where it was.
template <class R, bool GRAD>
constexpr int kWinDiag = (GRAD && sizeof(R) == 8) ? 128 : 256;

// acc[k] = sum_d B[l][d] v_k[64 blk + dlo + d + l], k < NC, for one 64-row
// block of a band in diagonal layout (entry (l, d) at off + (d - dlo) * 64 + l),
// each summed over d in ascending order.  Entry c of vector k (0 <= c < n;
// the vectors are 0 elsewhere) is the sum of the C chunk partials
// sc[(chunk*5 + k)*n + c]; the entries are staged
// per wavefront in LDS ([NC][64 + WD + kTailBatch]: a window plus zeros that
// the last, partial batch of diagonals reads), WD diagonals at a time.
template <class R, int NC, int WD>
__device__ __forceinline__ void band_block_dot(const R* __restrict__ Bv, const SliceDev& sd,
                                               int blk, int lane, int n, R* win,
                                               const R* __restrict__ sc, int C, R (&acc)[NC]) {
  constexpr int WS = kSlice + WD + kTailBatch<R>;
  const R* bv = Bv + sd.off + lane;
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = R(0);
  for (int d0 = 0; d0 < sd.nd; d0 += WD) {
    const int d1 = min(sd.nd, d0 + WD);
    // Window over the vector entries these diagonals touch: index
    // blk*64 + dlo + d0 + w, w < 64 + (d1 - d0) - 1.
    const int cbase = blk * kSlice + sd.dlo + d0;
    const int wn = kSlice + (d1 - d0) - 1;
    if (C == 1) {
      // One chunk: the entries are plain loads, all of two trips in flight.
#pragma unroll 2
      for (int w = lane; w < wn + kTailBatch<R>; w += kWave) {
        const int c = cbase + w;
        const bool in = w < wn && (unsigned)c < (unsigned)n;
        R v[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) v[k] = in ? sc[(int64_t)k * n + c] : R(0);
#pragma unroll
        for (int k = 0; k < NC; ++k) win[k * WS + w] = v[k];
      }
    } else {
      for (int w = lane; w < wn + kTailBatch<R>; w += kWave) {
        const int c = cbase + w;
        const bool in = w < wn && (unsigned)c < (unsigned)n;
        // One vector at a time: its chunk loads go out together, and the
        // registers stay free for the band loads below.
#pragma unroll 1
        for (int k = 0; k < NC; ++k) win[k * WS + w] = in ? sum_chunks<R>(sc, C, k, n, c) : R(0);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const R* wl = win + lane - d0;
    for (int d = d0; d < d1; d += kTailBatch<R>) {
      // The band loads go out together (the last, partial batch too: its
      // missing diagonals load nothing and add exact zeros); the window
      // reads (LDS) follow them.
      R x[kTailBatch<R>];
#pragma unroll
      for (int u = 0; u < kTailBatch<R>; ++u)
        x[u] = (d + u < d1) ? bv[(int64_t)(d + u) * kSlice] : R(0);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kTailBatch<R>; ++u)
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] = rfma<R>(x[u], wl[k * WS + d + u], acc[k]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// One slice of the tail of fit slice_prob[item]: its 64 rows of nu = norm R mu0
// (and R J0 with the gradient), their chi^2 terms and gradient seeds, summed
// over the wavefront; lane 0 stores the six partials at part[item].  Shared by
// the split tail and the queued tail, whose arguments (A) carry the same
// fields, so both give the same bits.
template <class R, bool GRAD, class A>
__device__ __forceinline__ void slice_tail(const A& a, int64_t item, int lane, R* win) {
  constexpr int NC = GRAD ? 5 : 1;
  constexpr int WD = kWinDiag<R, GRAD>;
  const int f = a.slice_prob[item];
  const ProbDev pd = a.probs[f];
  const int s = (int)(item - pd.slice_off);
  const int nb = pd.n_bins, C = pd.C;
  const R* sc = a.scratch + pd.scratch_off;
  const double norm = a.params[5 * (int64_t)f + 4];
  // acc[0] = (R mu0)_i and, with the gradient, acc[1 + c] = (R J0)_ic.
  R acc[NC];
  band_block_dot<R, NC, WD>(a.Rv, a.slices[item], s, lane, nb, win, sc, C, acc);
  const int i = s * kSlice + lane;
  double chi = 0.0;
  double gs[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  bool badnu = false;
  if (i < nb) {
    const double nu = norm * (double)acc[0];
    const double d = a.data[pd.bin_off + i];
    badnu = !(nu > 0.0) || !isfinite(nu);
    const double ratio = quot_pos(d, nu);
    chi = dfma(d, log_pos(d > 0.0 ? ratio : 1.0), nu - d);  // d = 0 takes ln 1 = 0
    if (GRAD) {
      const double gn = 2.0 * (1.0 - ratio);
#pragma unroll
      for (int c = 0; c < 4; ++c) gs[c] = gn * (double)acc[(1 + c) % NC];
      gs[4] = gn * (double)acc[0];
    }
    if (a.pred) a.pred[pd.bin_off + i] = nu;
  }
  if (badnu) __hip_atomic_fetch_or(a.status, (uint32_t)kBadPrediction, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
  chi = wave_total(chi);
  if (GRAD) {
#pragma unroll
    for (int c = 0; c < 5; ++c) gs[c] = wave_total(gs[c]);
  }
  if (lane == kWave - 1) {
    a.part[item * 6] = chi;
    if (GRAD) {
#pragma unroll
      for (int c = 0; c < 5; ++c) a.part[item * 6 + 1 + c] = gs[c];
    }
  }
}

template <class R, bool GRAD>
__global__ void __launch_bounds__(kTailWaves * kWave) tail_fwd_kernel(TailArgs<R> a) {
  constexpr int NC = GRAD ? 5 : 1;
  constexpr int WD = kWinDiag<R, GRAD>;
  __shared__ R win_all[kTailWaves][NC * (kSlice + WD + kTailBatch<R>)];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x - (threadIdx.x / kWave) * kWave;
  const int64_t idx = (int64_t)blockIdx.x * kTailWaves + wave;
  if (idx >= a.n_items) return;  // whole wavefronts leave; no work-group barrier below
  slice_tail<R, GRAD>(a, a.order[idx], lane, win_all[wave]);
}

// The chi^2 and gradient of fit f from its slice partials: lane s takes slice
// s (a fit has at most kMaxBins / 64 = 64 of them), and the wavefront sums
// are fixed-order.  Shared by the split and the queued tail.
template <class R, bool GRAD, class A>
__device__ __forceinline__ void fit_final(const A& a, int f, int lane) {
  static_assert(kMaxBins <= kSlice * kWave, "one lane per slice");
  const ProbDev pd = a.probs[f];
  const double* th = a.params + 5 * (int64_t)f;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (lane < pd.n_slices) {
    const double* q = a.part + (pd.slice_off + lane) * 6;
#pragma unroll
    for (int c = 0; c < (GRAD ? 6 : 1); ++c) v[c] = q[c];
  }
#pragma unroll
  for (int c = 0; c < (GRAD ? 6 : 1); ++c) v[c] = wave_total(v[c]);
  if (lane != kWave - 1) return;
  const bool bad = pee_coef<R>(th).bad;
  if (bad) __hip_atomic_fetch_or(a.status, (uint32_t)kBadMixing, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
  a.chi2[f] = bad ? NAN : 2.0 * v[0];
  if (GRAD && a.grad) {
    const double norm = th[4];
    double* gp = a.grad + 5 * (int64_t)f;
#pragma unroll
    for (int c = 0; c < 4; ++c) gp[c] = bad ? NAN : norm * v[1 + c];
    gp[4] = bad ? NAN : v[5];
  }
}

// One wavefront per fit.
template <class R, bool GRAD>
__global__ void __launch_bounds__(kTailWaves * kWave) tail_final_kernel(TailArgs<R> a) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x - (threadIdx.x / kWave) * kWave;
  const int f = blockIdx.x * kTailWaves + wave;
  if (f >= a.n_fits) return;
  fit_final<R, GRAD>(a, f, lane);
}

// ---- queued tail (uneven batches, one persistent launch) --------------------
// The queue (built by the plan) interleaves the point tiles with one tail item
// per fit, each after all of its fit's tiles.  The work-group that takes fit
// f's tail waits until f's tiles have counted themselves done: each of them
// was handed out before, to a work-group that waits on nothing, so the wait
// ends (it is bounded all the same: past kSpinLimit sleeps the work-group
// latches kSpinTimeout and waits no more in this launch).  One agent-scope
// acquire then covers every bin sum of the fit; its wavefronts take the fit's
// 64-row slices in
// turn (the slice work of tail_fwd), and wavefront 0 adds the slice partials
// as tail_final does, after a work-group barrier.  The fit's data crosses
// work-groups once per fit, not once per slice (each crossing costs an L2
// write-back or invalidation on a GPU of several L2s).  Same operations in
// the same order as the split tail, so the results are the same bits.
constexpr uint32_t kSpinLimit = 1u << 20;  // >= 1M sleeps of 128 clocks: tens of ms at least

template <class R, bool GRAD>
__device__ void queued_fit(const ChainArgs<R>& a, int f, int wave, int nw, int lane, R* win,
                           uint32_t* late) {
  if (threadIdx.x == 0) {
    const uint32_t need = (uint32_t)(a.probs[f].n_bin_blocks * a.probs[f].C) + a.need_extra;
    uint32_t spin = 0;
    while (!*late &&
           __hip_atomic_load(&a.counters[f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
      if (++spin > a.spin_limit) {
        *late = 1u;
        __hip_atomic_fetch_or(a.status, (uint32_t)kSpinTimeout, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the fit's bin sums
    // Every tile of the fit has counted: the counter starts the next
    // evaluation at zero (the launch boundary publishes the store).
    a.counters[f] = 0u;
  }
  __syncthreads();
  const ProbDev pd = a.probs[f];
  for (int s = wave; s < pd.n_slices; s += nw) slice_tail<R, GRAD>(a, pd.slice_off + s, lane, win);
  __syncthreads();  // the slice partials of every wavefront
  if (wave == 0) fit_final<R, GRAD>(a, f, lane);
}

// Window LDS of one wavefront of the queued tail.
template <class R, bool GRAD>
constexpr int kQueuedWin = (GRAD ? 5 : 1) * (kSlice + kWinDiag<R, GRAD> + kTailBatch<R>);

}  // namespace

size_t queued_lds_bytes(const gna_plan* p, const Shape& sh) {
  const size_t per_wave = p->prec == GNA_FP64 ? sizeof(double) * kQueuedWin<double, true>
                                              : sizeof(float) * kQueuedWin<float, true>;
  return (size_t)(sh.threads / kWave) * per_wave;
}

namespace {

template <class R, bool GRAD>
__global__ void __launch_bounds__(1024) chain_queued_kernel(ChainArgs<R> a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ BaseLds bl;
  __shared__ uint32_t next;
  __shared__ uint32_t late;  // set when a wait gave up (the rest of the launch does not wait)
  const int nw = blockDim.x / kWave;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x - (threadIdx.x / kWave) * kWave;
  TileLds L{lds_raw, (int)blockDim.x, 0, 1};
  if (threadIdx.x == 0) late = 0u;
  for (;;) {
    if (threadIdx.x == 0)
      next = __hip_atomic_fetch_add(&a.queue[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t t = next;
    __syncthreads();
    if (t >= a.n_items) break;
    const int32_t e = a.q_items[t];
    if (e >= 0)
      process_tile<R, GRAD, true, true>(a, e, L, bl);
    else
      queued_fit<R, GRAD>(a, -1 - e, wave, nw, lane,
                          reinterpret_cast<R*>(lds_raw) + (size_t)wave * kQueuedWin<R, GRAD>,
                          &late);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint32_t done = __hip_atomic_fetch_add(&a.queue[1], 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (done + 1 == gridDim.x) {
      a.queue[0] = 0u;
      a.queue[1] = 0u;
    }
  }
}

template <class R>
int launch_tail(gna_plan* p, const ChainArgs<R>& c, bool grad, hipStream_t s) {
  unsigned char* w = p->ws;
  TailArgs<R> a{};
  a.probs = c.probs;
  a.slices = c.slices;
  a.slice_prob = (const int32_t*)(w + p->lay.slice_prob);
  a.order = (const int32_t*)(w + p->lay.fwd_order);
  a.n_items = p->total_slices;
  a.n_fits = p->n_points;
  a.Rv = c.Rv;
  a.data = c.data;
  a.params = c.params;
  a.scratch = c.scratch;
  a.part = (double*)(w + p->lay.tailpart);
  a.pred = c.pred;
  a.status = c.status;
  a.chi2 = c.chi2;
  a.grad = c.grad;
  const unsigned g = (unsigned)((a.n_items + kTailWaves - 1) / kTailWaves);
  const unsigned gf = (unsigned)((a.n_fits + kTailWaves - 1) / kTailWaves);
  const dim3 blk(kTailWaves * kWave);
  if (grad) {
    hipLaunchKernelGGL((tail_fwd_kernel<R, true>), dim3(g), blk, 0, s, a);
    hipLaunchKernelGGL((tail_final_kernel<R, true>), dim3(gf), blk, 0, s, a);
  } else {
    hipLaunchKernelGGL((tail_fwd_kernel<R, false>), dim3(g), blk, 0, s, a);
    hipLaunchKernelGGL((tail_final_kernel<R, false>), dim3(gf), blk, 0, s, a);
  }
  return check_hip(hipGetLastError(), "tail kernel launch");
}

template <class R, bool GRAD, bool PERSIST, bool SPLIT>
int launch_t(gna_plan* p, const ChainArgs<R>& a, hipStream_t s) {
  const Shape& sh = p->shape;
  auto kern = chain_kernel<R, GRAD, PERSIST, SPLIT>;
  gna_plan::LaunchCache& lc = p->launch_cache[GRAD];
  if (!lc.ready) {
    lc.lds = chain_lds_bytes(p, sh);
    lc.occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&lc.occ, kern, sh.threads, lc.lds) !=
            hipSuccess ||
        lc.occ < 1)
      lc.occ = 1;
    lc.share = 0;
    lc.rlds = 0;
    lc.ready = 1;
  }
  const size_t lds = lc.lds;
  int64_t grid = a.n_tiles;
  if (PERSIST) grid = std::min<int64_t>(a.n_tiles, (int64_t)lc.occ * p->cu_count);
  if (grid < 1) return GNA_OK;
  if (grid > 0x7fffffffLL / sh.threads)
    return fail(GNA_E_UNSUPPORTED, "%lld tiles exceed one launch; use the persistent shape",
                (long long)grid);
  const ChainLds cl = chain_lds(p, sh);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(sh.threads), lds, s, a, cl.vs, cl.kf_cap);
  return check_hip(hipGetLastError(), "chain_kernel launch");
}

template <class R>
int launch_point_tails(gna_plan* p, const ChainArgs<R>& a, int32_t B, bool grad, hipStream_t s) {
  Shape ts = p->shape;
  ts.threads = kChainTailThreads;
  const ChainLds cl = chain_lds(p, ts);  // the fused tail's layout at the tail's width
  if (grad)
    hipLaunchKernelGGL((chain_tail_kernel<R, true>), dim3((unsigned)B), dim3(kChainTailThreads),
                       cl.bytes, s, a, cl.vs, cl.kf_cap);
  else
    hipLaunchKernelGGL((chain_tail_kernel<R, false>), dim3((unsigned)B), dim3(kChainTailThreads),
                       cl.bytes, s, a, cl.vs, cl.kf_cap);
  return check_hip(hipGetLastError(), "chain_tail_kernel launch");
}

template <class R, bool GRAD>
int launch_queued(gna_plan* p, const ChainArgs<R>& a, hipStream_t s) {
  const Shape& sh = p->shape;
  auto kern = chain_queued_kernel<R, GRAD>;
  gna_plan::LaunchCache& lc = p->launch_cache[GRAD];
  if (!lc.ready) {
    lc.lds = queued_lds_bytes(p, sh);
    if (lc.lds > 64 * 1024) {
      const int rc = check_hip(hipFuncSetAttribute((const void*)kern,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)lc.lds),
                               "hipFuncSetAttribute (queued-tail LDS)");
      if (rc) return rc;
    }
    lc.occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&lc.occ, kern, sh.threads, lc.lds) !=
            hipSuccess ||
        lc.occ < 1)
      lc.occ = 1;
    lc.share = 0;
    lc.rlds = 0;
    lc.ready = 1;
  }
  const int64_t grid = std::min<int64_t>(a.n_items, (int64_t)lc.occ * p->cu_count);
  if (grid < 1) return GNA_OK;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(sh.threads), lc.lds, s, a);
  return check_hip(hipGetLastError(), "chain_queued_kernel launch");
}

template <class R>
int launch_r(gna_plan* p, const double* params, int32_t B, double* chi2, double* grad,
             double* pred, hipStream_t s, const double* host_params) {
  unsigned char* w = p->ws;
  const Layout& L = p->lay;
  ChainArgs<R> a{};
  if (!params) {
    if (B != 1 || !host_params || p->kind != kChain)
      return fail(GNA_E_INVAL, "parameters by value: one point of a chain plan only");
    for (int c = 0; c < 5; ++c) a.pin[c] = host_params[c];
  }
  a.probs = (const ProbDev*)(w + L.probs);
  if (p->kind == kChain) {
    a.tiles = nullptr;
    a.tiles_per_point = (int32_t)p->n_tiles;
    a.n_tiles = (int64_t)B * p->n_tiles;
    a.scratch_stride = (int64_t)p->ccap * 5 * p->probs[0].n_bins;
  } else {
    a.tiles = (const TileDev*)(w + L.tiles);
    a.tiles_per_point = 0;
    a.n_tiles = p->n_tiles;
    a.scratch_stride = 0;
  }
  a.want_grad = grad ? 1 : 0;
  a.E = (const double*)(w + L.E);
  a.f = (const R*)(w + L.f);
  a.L = (const double*)(w + L.L);
  a.wL = (const double*)(w + L.wL);
  a.data = (const double*)(w + L.data);
  a.slices = (const SliceDev*)(w + L.slices);
  a.Rv = (const R*)(w + L.Rv);
  a.params = params;
  a.scratch = (R*)(w + L.scratch);
  a.counters = (uint32_t*)(w + L.counters);
  a.status = (uint32_t*)(w + L.status);
  a.queue = (uint32_t*)(w + L.queue);
  a.chi2 = chi2;
  a.grad = grad;
  a.pred = pred;
  const bool pers = p->shape.persistent != 0;
  if (p->shape.split == 2) {
    a.q_items = (const int32_t*)(w + L.q_items);
    a.n_items = p->n_qitems;
    a.slice_prob = (const int32_t*)(w + L.slice_prob);
    a.part = (double*)(w + L.tailpart);
    a.spin_limit = p->q_spin_limit ? p->q_spin_limit : kSpinLimit;
    a.need_extra = p->q_need_extra;
    return grad ? launch_queued<R, true>(p, a, s) : launch_queued<R, false>(p, a, s);
  }
  if (p->shape.split) {
    int rc;
    if (grad)
      rc = pers ? launch_t<R, true, true, true>(p, a, s) : launch_t<R, true, false, true>(p, a, s);
    else
      rc = pers ? launch_t<R, false, true, true>(p, a, s) : launch_t<R, false, false, true>(p, a, s);
    if (rc) return rc;
    if (p->kind == kChain) return launch_point_tails<R>(p, a, B, grad != nullptr, s);
    return launch_tail<R>(p, a, grad != nullptr, s);
  }
  if (grad) {
    return pers ? launch_t<R, true, true, false>(p, a, s) : launch_t<R, true, false, false>(p, a, s);
  }
  return pers ? launch_t<R, false, true, false>(p, a, s) : launch_t<R, false, false, false>(p, a, s);
}

}  // namespace

int launch_chain(gna_plan* p, const double* params, int32_t B, double* chi2, double* grad,
                 double* pred, hipStream_t s, const double* host_params) {
  if (p->prec == GNA_FP64) return launch_r<double>(p, params, B, chi2, grad, pred, s, host_params);
  return launch_r<float>(p, params, B, chi2, grad, pred, s, host_params);
}

}  // namespace gna

extern "C" int gna_debug_queued_wait(gna_plan* plan, int32_t spin_limit, int32_t extra_tiles) {
  gna::clear_error();
  if (!plan) return gna::fail(GNA_E_INVAL, "plan is NULL");
  if (plan->kind != gna::kFitset)
    return gna::fail(GNA_E_INVAL, "gna_debug_queued_wait: not a fitset plan");
  if (spin_limit < 0 || extra_tiles < 0)
    return gna::fail(GNA_E_INVAL, "gna_debug_queued_wait: spin_limit %d, extra_tiles %d < 0",
                     spin_limit, extra_tiles);
  plan->q_spin_limit = (uint32_t)spin_limit;
  plan->q_need_extra = (uint32_t)extra_tiles;
  return GNA_OK;
}
