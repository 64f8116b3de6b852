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
// Tail (one work-group per point):
//   nu_i    = sum_j R_ij mu_j          banded R, one wavefront per 64-row slice
//   chi2    = 2 sum_i [nu_i - d_i + d_i ln(d_i / nu_i)]     (FP64)
//   gnu_i   = 2 (1 - d_i / nu_i)                            (FP64, stored in R)
//   gmu_j   = sum_i R_ij gnu_i         the same band, walked by columns
//   grad_c  = norm sum_j gmu_j J0_jc,  grad_norm = sum_j gmu_j mu0_j   (FP64 sums)
#include <cmath>

#include "gna_internal.h"
#include "gna_math.h"

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

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Dynamic LDS of one work-group (sizes in chain_lds_bytes):
//   stage [threads][5]        bin sums of a single-tile point
//   mu    [max_bins]          norm * mu0
//   gnu   [max_bins]          d chi2 / d nu
//   part  [split][max_bins]   partial smearing sums of the diagonal chunks
//                             (absent when split == 1: the forward partials
//                             then live in gnu, read and overwritten element
//                             by element, and the adjoint partials in mu,
//                             which the adjoint no longer reads)
//   red   [waves][6]          per-wave chi2 and gradient partials
//   flag
struct TileLds {
  unsigned char* base;
  int threads;
  int max_bins;
  int split;
  __device__ static size_t align16(size_t x) { return (x + 15) & ~size_t(15); }
  template <class R>
  __device__ size_t o_mu() const { return align16((size_t)threads * 5 * sizeof(R)); }
  template <class R>
  __device__ size_t o_gnu() const { return o_mu<R>() + align16((size_t)max_bins * sizeof(R)); }
  template <class R>
  __device__ size_t o_part() const { return o_gnu<R>() + align16((size_t)max_bins * sizeof(R)); }
  template <class R>
  __device__ size_t o_red() const {
    return o_part<R>() + (split > 1 ? align16((size_t)split * max_bins * sizeof(R)) : 0);
  }
  template <class R>
  __device__ R* stage() const { return reinterpret_cast<R*>(base); }
  template <class R>
  __device__ R* mu() const { return reinterpret_cast<R*>(base + o_mu<R>()); }
  template <class R>
  __device__ R* gnu() const { return reinterpret_cast<R*>(base + o_gnu<R>()); }
  template <class R>
  __device__ R* part_fwd() const {
    return split > 1 ? reinterpret_cast<R*>(base + o_part<R>()) : gnu<R>();
  }
  template <class R>
  __device__ R* part_adj() const {
    return split > 1 ? reinterpret_cast<R*>(base + o_part<R>()) : mu<R>();
  }
  template <class R>
  __device__ double* red() const { return reinterpret_cast<double*>(base + o_red<R>()); }
  template <class R>
  __device__ int* flag() const { return reinterpret_cast<int*>(red<R>() + (threads / kWave) * 6); }
};

// gmu_j = sum_i R_ij gnu_i over diagonals d in [d0, d1), for the 64 columns
// j = 64 cb + lane.  Row i = j - d lies in slice cb - m (lanes >= r) or
// cb - m - 1 (lanes < r), with d = 64 m + r: every lane is busy and each
// slice is read as one contiguous segment.  Branch-free body (invalid lanes
// read element 0 and add 0) so the unrolled loads issue back to back.
template <class R>
__device__ R adjoint_range(const R* __restrict__ Rv, const SliceDev* __restrict__ slices, int ns,
                           int nb, const R* gnus, int cb, int lane, int d0, int d1) {
  R acc = R(0);
  int d = d0;
  while (d < d1) {
    const int m = d >> 6;  // floor(d / 64)
    const int dend = min(d1, (m + 1) * kSlice);
    const int sB = cb - m, sA = cb - m - 1;
    const bool vB = sB >= 0 && sB < ns, vA = sA >= 0 && sA < ns;
    const SliceDev zB = vB ? slices[sB] : SliceDev{0, 0, 0};
    const SliceDev zA = vA ? slices[sA] : SliceDev{0, 0, 0};
    auto term = [&](int dd, R& rv, R& g) {
      const int r = dd - m * kSlice;
      const bool useB = lane >= r;
      const int s = useB ? sB : sA;
      const int dlo = useB ? zB.dlo : zA.dlo;
      const int nd = useB ? zB.nd : zA.nd;
      const int64_t off = useB ? zB.off : zA.off;
      const int li = useB ? lane - r : lane + kSlice - r;
      const int i = s * kSlice + li;
      const bool ok = (dd >= dlo) && (dd < dlo + nd) && (i < nb);
      const R x = Rv[ok ? off + (int64_t)(dd - dlo) * kSlice + li : 0];
      const R y = gnus[ok ? i : 0];
      rv = ok ? x : R(0);
      g = y;
    };
    // Batches of kTailBatch loads issued together (the barrier keeps the
    // scheduler from pairing each load with its FMA); same summation order.
    for (; d + kTailBatch<R> <= dend; d += kTailBatch<R>) {
      R x[kTailBatch<R>], y[kTailBatch<R>];
#pragma unroll
      for (int u = 0; u < kTailBatch<R>; ++u) term(d + u, x[u], y[u]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kTailBatch<R>; ++u) acc = rfma<R>(x[u], y[u], acc);
    }
    for (; d < dend; ++d) {
      R x, y;
      term(d, x, y);
      acc = rfma<R>(x, y, acc);
    }
  }
  return acc;
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

// Baseline constants of the current tile's problem, staged once per tile so
// the per-baseline loop reads LDS (a broadcast) instead of waiting on memory.
struct BaseLds {
  double kl[kMaxBaselines];  // K L_r
  double w[kMaxBaselines];   // w_r
};

template <class R, bool GRAD, bool SPLIT>
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
  const double* th = a.params + 5 * (int64_t)td.point;
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
  for (int off = G >> 1; off > 0; off >>= 1) {
    mu += __shfl_xor(mu, off, kWave);
    if (GRAD) {
#pragma unroll
      for (int c = 0; c < 4; ++c) J[c] += __shfl_xor(J[c], off, kWave);
    }
  }

  const int nb = pd.n_bins;
  if (SPLIT) {
    // Split tail: every tile leaves its partial sums in the scratch region;
    // the tail kernels read them after this launch.
    R* sc = a.scratch + pd.scratch_off;
    if (g == 0 && lb < pd.bins_per_tile && j < nb) {
      sc[(int64_t)(td.chunk * 5) * nb + j] = mu;
      if (GRAD) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sc[(int64_t)(td.chunk * 5 + 1 + c) * nb + j] = J[c];
      }
    }
    return;
  }
  const int tiles_of_point = pd.n_bin_blocks * pd.C;
  const bool single = (tiles_of_point == 1);
  R* stage = L.stage<R>();
  R* sc = a.scratch + (a.tiles ? pd.scratch_off : (int64_t)td.point * a.scratch_stride);
  if (g == 0 && lb < pd.bins_per_tile && j < nb) {
    if (single) {
      stage[lb * 5] = mu;
      if (GRAD) {
#pragma unroll
        for (int c = 0; c < 4; ++c) stage[lb * 5 + 1 + c] = J[c];
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

  // ---- tail ----------------------------------------------------------------
  const int C = pd.C;
  auto mu0_of = [&](int jj) -> R {
    return single ? stage[jj * 5] : sum_chunks<R>(sc, C, 0, nb, jj);
  };
  auto J0_of = [&](int jj, int cidx) -> R {
    return single ? stage[jj * 5 + 1 + cidx] : sum_chunks<R>(sc, C, 1 + cidx, nb, jj);
  };
  const double norm = th[4];
  const R normr = (R)norm;
  R* mus = L.mu<R>();
  R* gnus = L.gnu<R>();
  for (int jj = tid; jj < nb; jj += NT) mus[jj] = normr * mu0_of(jj);
  __syncthreads();

  const int wave = tid / kWave, lane = tid - (tid / kWave) * kWave;
  const int nwaves = NT / kWave;
  const int ns = pd.n_slices;
  const SliceDev* slices = a.slices + pd.slice_off;
  const double* dat = a.data + pd.bin_off;
  double* pred = a.pred ? (a.tiles ? a.pred + pd.bin_off : a.pred + (int64_t)td.point * nb)
                        : nullptr;
  R* part = L.part_fwd<R>();
  const int maxb = L.max_bins;

  // Forward smearing: work items (slice, chunk of its diagonals) over all waves.
  const int Kf = min(L.split, max(1, nwaves / ns));
  for (int item = wave; item < ns * Kf; item += nwaves) {
    const int s = item / Kf, kap = item - (item / Kf) * Kf;
    const SliceDev sd = slices[s];
    const int csz = (sd.nd + Kf - 1) / Kf;
    const int d0 = kap * csz, d1 = min(sd.nd, d0 + csz);
    const int i = s * kSlice + lane;
    const R* rv = a.Rv + sd.off + lane;
    auto term = [&](int dd, R& x, R& y) {
      const int jj = i + sd.dlo + dd;
      const R m = mus[((unsigned)jj < (unsigned)nb) ? jj : 0];
      x = rv[(int64_t)dd * kSlice];
      y = ((unsigned)jj < (unsigned)nb) ? m : R(0);
    };
    R acc = R(0);
    int dd = d0;
    for (; dd + kTailBatch<R> <= d1; dd += kTailBatch<R>) {
      R x[kTailBatch<R>], y[kTailBatch<R>];
#pragma unroll
      for (int u = 0; u < kTailBatch<R>; ++u) term(dd + u, x[u], y[u]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kTailBatch<R>; ++u) acc = rfma<R>(x[u], y[u], acc);
    }
    for (; dd < d1; ++dd) {
      R x, y;
      term(dd, x, y);
      acc = rfma<R>(x, y, acc);
    }
    if (i < nb) part[kap * maxb + i] = acc;
  }
  __syncthreads();
  double chi = 0.0;
  bool badnu = false;
  for (int i = tid; i < nb; i += NT) {
    R acc = R(0);
    for (int kap = 0; kap < Kf; ++kap) acc += part[kap * maxb + i];
    const double nu = (double)acc;
    const double d = dat[i];
    if (!(nu > 0.0) || !isfinite(nu)) badnu = true;
    const double ratio = quot_pos(d, nu);
    chi += dfma(d, log_pos(d > 0.0 ? ratio : 1.0), nu - d);  // d = 0 takes ln 1 = 0
    gnus[i] = (R)(2.0 * (1.0 - ratio));
    if (pred) pred[i] = nu;
  }
  if (badnu) __hip_atomic_fetch_or(a.status, (uint32_t)kBadPrediction, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
  double* red = L.red<R>();
  chi = wave_sum(chi);
  if (lane == 0) red[wave * 6] = chi;
  __syncthreads();

  double gs[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (GRAD) {
    part = L.part_adj<R>();
    // Adjoint smearing: work items (column block, chunk of its diagonals).
    const int ncb = (nb + kSlice - 1) / kSlice;
    const int Ka = min(L.split, max(1, nwaves / ncb));
    for (int item = wave; item < ncb * Ka; item += nwaves) {
      const int cb = item / Ka, kap = item - (item / Ka) * Ka;
      int dmin = 1 << 30, dmax = -(1 << 30);
      for (int s = 0; s < ns; ++s) {
        const SliceDev sd = slices[s];
        const int lo = max(sd.dlo, kSlice * (cb - s) - (kSlice - 1));
        const int hi = min(sd.dlo + sd.nd - 1, kSlice * (cb - s) + (kSlice - 1));
        if (lo <= hi) {
          dmin = min(dmin, lo);
          dmax = max(dmax, hi);
        }
      }
      R acc = R(0);
      if (dmin <= dmax) {
        const int span = dmax - dmin + 1;
        const int csz = (span + Ka - 1) / Ka;
        const int d0 = dmin + kap * csz, d1 = min(dmax + 1, d0 + csz);
        acc = adjoint_range<R>(a.Rv, slices, ns, nb, gnus, cb, lane, d0, d1);
      }
      const int jc = cb * kSlice + lane;
      if (jc < nb) part[kap * maxb + jc] = acc;
    }
    __syncthreads();
    for (int jc = tid; jc < nb; jc += NT) {
      R acc = R(0);
      for (int kap = 0; kap < Ka; ++kap) acc += part[kap * maxb + jc];
      const double gmu = (double)acc;
#pragma unroll
      for (int c = 0; c < 4; ++c) gs[c] += gmu * (double)J0_of(jc, c);
      gs[4] += gmu * (double)mu0_of(jc);
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) gs[c] = wave_sum(gs[c]);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < 5; ++c) red[wave * 6 + 1 + c] = gs[c];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double chisum = 0.0, g5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < nwaves; ++w) {
      chisum += red[w * 6];
      if (GRAD) {
#pragma unroll
        for (int c = 0; c < 5; ++c) g5[c] += red[w * 6 + 1 + c];
      }
    }
    const bool bad = k.bad;
    if (bad) __hip_atomic_fetch_or(a.status, (uint32_t)kBadMixing, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    a.chi2[td.point] = bad ? NAN : 2.0 * chisum;
    if (GRAD && a.grad) {
      double* gp = a.grad + 5 * (int64_t)td.point;
#pragma unroll
      for (int c = 0; c < 4; ++c) gp[c] = bad ? NAN : norm * g5[c];
      gp[4] = bad ? NAN : g5[4];
    }
  }
}

template <class R, bool GRAD, bool PERSIST, bool SPLIT>
__global__ void __launch_bounds__(1024) chain_kernel(ChainArgs<R> a, int max_bins, int split) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  TileLds L{lds_raw, (int)blockDim.x, max_bins, split};
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
// each summed over d in ascending order.  vat(c, k) gives entry c of vector
// k for 0 <= c < n (the vectors are 0 elsewhere); they are staged
// per wavefront in LDS ([NC][64 + WD]), WD diagonals at a time.
template <class R, int NC, int WD, class V>
__device__ __forceinline__ void band_block_dot(const R* __restrict__ Bv, const SliceDev& sd,
                                               int blk, int lane, int n, R* win, V vat,
                                               R (&acc)[NC]) {
  constexpr int WS = kSlice + WD;
  const R* bv = Bv + sd.off + lane;
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = R(0);
  for (int d0 = 0; d0 < sd.nd; d0 += WD) {
    const int d1 = min(sd.nd, d0 + WD);
    // Window over the vector entries these diagonals touch: index
    // blk*64 + dlo + d0 + w, w < 64 + (d1 - d0) - 1.
    const int cbase = blk * kSlice + sd.dlo + d0;
    const int wn = kSlice + (d1 - d0) - 1;
    for (int w = lane; w < wn; w += kWave) {
      const int c = cbase + w;
      const bool in = (unsigned)c < (unsigned)n;
      // One vector at a time: its loads go out together, and the registers
      // stay free for the band loads below.
#pragma unroll 1
      for (int k = 0; k < NC; ++k) win[k * WS + w] = in ? vat(c, k) : R(0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const R* wl = win + lane - d0;
    int d = d0;
    for (; d + kTailBatch<R> <= d1; d += kTailBatch<R>) {
      // The band loads go out together; the window reads (LDS) follow them.
      R x[kTailBatch<R>];
#pragma unroll
      for (int u = 0; u < kTailBatch<R>; ++u) x[u] = bv[(int64_t)(d + u) * kSlice];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kTailBatch<R>; ++u)
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] = rfma<R>(x[u], wl[k * WS + d + u], acc[k]);
    }
    for (; d < d1; ++d) {
      const R x = bv[(int64_t)d * kSlice];
#pragma unroll
      for (int k = 0; k < NC; ++k) acc[k] = rfma<R>(x, wl[k * WS + d], acc[k]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <class R, bool GRAD>
__global__ void __launch_bounds__(kTailWaves * kWave) tail_fwd_kernel(TailArgs<R> a) {
  constexpr int NC = GRAD ? 5 : 1;
  constexpr int WD = kWinDiag<R, GRAD>;
  __shared__ R win_all[kTailWaves][NC * (kSlice + WD)];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x - (threadIdx.x / kWave) * kWave;
  const int64_t idx = (int64_t)blockIdx.x * kTailWaves + wave;
  if (idx >= a.n_items) return;  // whole wavefronts leave; no work-group barrier below
  const int64_t item = a.order[idx];
  const int f = a.slice_prob[item];
  const ProbDev pd = a.probs[f];
  const int s = (int)(item - pd.slice_off);
  const int nb = pd.n_bins, C = pd.C;
  const R* sc = a.scratch + pd.scratch_off;
  const double norm = a.params[5 * (int64_t)f + 4];
  // acc[0] = (R mu0)_i and, with the gradient, acc[1 + c] = (R J0)_ic.
  R acc[NC];
  band_block_dot<R, NC, WD>(a.Rv, a.slices[item], s, lane, nb, win_all[wave],
                            [&](int c, int k) { return sum_chunks<R>(sc, C, k, nb, c); }, acc);
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
  chi = wave_sum(chi);
  if (GRAD) {
#pragma unroll
    for (int c = 0; c < 5; ++c) gs[c] = wave_sum(gs[c]);
  }
  if (lane == 0) {
    a.part[item * 6] = chi;
    if (GRAD) {
#pragma unroll
      for (int c = 0; c < 5; ++c) a.part[item * 6 + 1 + c] = gs[c];
    }
  }
}

// One wavefront per fit: lane s takes slice s (a fit has at most
// kMaxBins / 64 = 64 of them), and the butterfly sums are fixed-order.
template <class R, bool GRAD>
__global__ void __launch_bounds__(kTailWaves * kWave) tail_final_kernel(TailArgs<R> a) {
  static_assert(kMaxBins <= kSlice * kWave, "one lane per slice");
  const int wave = threadIdx.x / kWave, lane = threadIdx.x - (threadIdx.x / kWave) * kWave;
  const int f = blockIdx.x * kTailWaves + wave;
  if (f >= a.n_fits) return;
  const ProbDev pd = a.probs[f];
  const double* th = a.params + 5 * (int64_t)f;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (lane < pd.n_slices) {
    const double* q = a.part + (pd.slice_off + lane) * 6;
#pragma unroll
    for (int c = 0; c < (GRAD ? 6 : 1); ++c) v[c] = q[c];
  }
#pragma unroll
  for (int c = 0; c < (GRAD ? 6 : 1); ++c) v[c] = wave_sum(v[c]);
  if (lane != 0) return;
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
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(sh.threads), lds, s, a, p->max_bins,
                     chain_split(p, sh));
  return check_hip(hipGetLastError(), "chain_kernel launch");
}

template <class R>
int launch_r(gna_plan* p, const double* params, int32_t B, double* chi2, double* grad,
             double* pred, hipStream_t s) {
  unsigned char* w = p->ws;
  const Layout& L = p->lay;
  ChainArgs<R> a{};
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
  if (p->shape.split) {
    int rc;
    if (grad)
      rc = pers ? launch_t<R, true, true, true>(p, a, s) : launch_t<R, true, false, true>(p, a, s);
    else
      rc = pers ? launch_t<R, false, true, true>(p, a, s) : launch_t<R, false, false, true>(p, a, s);
    if (rc) return rc;
    return launch_tail<R>(p, a, grad != nullptr, s);
  }
  if (grad) {
    return pers ? launch_t<R, true, true, false>(p, a, s) : launch_t<R, true, false, false>(p, a, s);
  }
  return pers ? launch_t<R, false, true, false>(p, a, s) : launch_t<R, false, false, false>(p, a, s);
}

}  // namespace

int launch_chain(gna_plan* p, const double* params, int32_t B, double* chi2, double* grad,
                 double* pred, hipStream_t s) {
  if (p->prec == GNA_FP64) return launch_r<double>(p, params, B, chi2, grad, pred, s);
  return launch_r<float>(p, params, B, chi2, grad, pred, s);
}

}  // namespace gna
