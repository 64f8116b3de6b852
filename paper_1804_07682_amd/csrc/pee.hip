// Elementwise survival probability over a resident energy vector (Sec. 4.1):
// P[i] = sum_r w_r P_ee(E[i]; L_r, theta).
//
// HBM-streaming kernel: 16-byte non-temporal loads of two energies per lane
// and 16-byte (FP64) or 8-byte (mixed) stores, software-pipelined; the probability needs only
// cos^2 of each phase, so one sin^2 polynomial per phase is evaluated
// (cos^2 = 1 - sin^2 >= 1/2 on the reduced argument).  Phases and their
// reduction are FP64 in both modes; q = KL / E comes from a refined
// reciprocal (correctly rounded in FP64 mode, ~2 ulp in mixed mode).
#include <algorithm>
#include <cmath>

#include "gna_internal.h"
#include "gna_math.h"

namespace gna {
namespace {

constexpr int kPeeThreads = 256;

template <class R>
struct PeeArgs {
  R K0, A, B1, B2;
  double dm21, dm31, dm32;
  int32_t n_L;
  double KL[kMaxBaselines];  // K * L_r, rounded once (the q = (K L) / E order)
  R w[kMaxBaselines];
};

template <class R, bool ONE_L>
__device__ __forceinline__ R pee_eval(const PeeArgs<R>& a, double E) {
  R acc = R(0);
  const int nL = ONE_L ? 1 : a.n_L;
  for (int r = 0; r < nL; ++r) {
    const double q = (sizeof(R) == 8) ? phase_per_ev2(a.KL[r], E) : phase_per_ev2_fast(a.KL[r], E);
    const R c21 = cos2_phase<R>(a.dm21 * q);
    const R c31 = cos2_phase<R>(a.dm31 * q);
    const R c32 = cos2_phase<R>(a.dm32 * q);
    R p = rfma_t<R>(a.A, c21, a.K0);
    p = rfma_t<R>(a.B1, c31, p);
    p = rfma_t<R>(a.B2, c32, p);
    acc = ONE_L ? p : acc + a.w[r] * p;
  }
  return acc;  // NaN for E <= 0 (see recip_pos)
}

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));

template <class R>
struct Vec2;
template <>
struct Vec2<double> {
  using T = dvec2;
};
template <>
struct Vec2<float> {
  using T = fvec2;
};

// Two ways of walking the pairs (E[2p], E[2p+1]), both software-pipelined:
// each lane issues the load of its next pair before evaluating the current
// one, so HBM traffic overlaps the arithmetic.
//  * grid-stride (mixed precision): pairs p, p + stride, ... with a grid of
//    256 work-groups per CU;
//  * chunked (FP64, whose evaluation is about twice as long): work-group b
//    owns the contiguous pairs [b C, (b + 1) C) and its lanes stride by the
//    group size, so each group streams one contiguous region.
// Both measured on MI355X against a streaming copy of the same size.
constexpr int64_t kPeeChunk = 2048;  // pairs per work-group in the chunked walk

template <class R, bool ONE_L>
__device__ __forceinline__ typename Vec2<R>::T pee_pair(const PeeArgs<R>& a, dvec2 e) {
  typename Vec2<R>::T o;
  o.x = pee_eval<R, ONE_L>(a, e.x);
  o.y = pee_eval<R, ONE_L>(a, e.y);
  return o;
}

// Pairs p0, p0 + step, ... below p1, pipelined.
template <class R, bool ONE_L>
__device__ __forceinline__ void pee_walk(const dvec2* __restrict__ E2,
                                         typename Vec2<R>::T* __restrict__ P2,
                                         const PeeArgs<R>& a, int64_t p0, int64_t p1,
                                         int64_t step) {
  if (p0 >= p1) return;
  dvec2 cur = __builtin_nontemporal_load(E2 + p0);
  for (int64_t p = p0;; p += step) {
    const int64_t nx = p + step;
    dvec2 nxt = cur;
    if (nx < p1) nxt = __builtin_nontemporal_load(E2 + nx);
    __builtin_nontemporal_store(pee_pair<R, ONE_L>(a, cur), P2 + p);
    if (nx >= p1) break;
    cur = nxt;
  }
}

template <class R, bool ONE_L, bool CHUNKED>
__global__ void __launch_bounds__(kPeeThreads)
    pee_kernel(const double* __restrict__ E, int64_t n, PeeArgs<R> a, R* __restrict__ P) {
  using V = typename Vec2<R>::T;
  const int64_t npairs = n >> 1;
  const dvec2* E2 = reinterpret_cast<const dvec2*>(E);
  V* P2 = reinterpret_cast<V*>(P);
  if (CHUNKED) {
    const int64_t b0 = (int64_t)blockIdx.x * kPeeChunk;
    const int64_t b1 = b0 + kPeeChunk < npairs ? b0 + kPeeChunk : npairs;
    pee_walk<R, ONE_L>(E2, P2, a, b0 + threadIdx.x, b1, kPeeThreads);
  } else {
    pee_walk<R, ONE_L>(E2, P2, a, (int64_t)blockIdx.x * kPeeThreads + threadIdx.x, npairs,
                       (int64_t)gridDim.x * kPeeThreads);
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) P[n - 1] = pee_eval<R, ONE_L>(a, E[n - 1]);
}

int g_cu_count = 0;

int cu_count() {
  if (g_cu_count > 0) return g_cu_count;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  g_cu_count = cus;
  return cus;
}

template <class R>
int run_pee(const double* E, int64_t n, int32_t n_L, const double* L, const double* wL,
            const double* th, void* P, hipStream_t s) {
  PeeArgs<R> a{};
  const double s12 = th[2], s13 = th[3];
  const double c12 = 1.0 - s12, c13 = 1.0 - s13;
  const double A = 4.0 * s12 * c12 * (c13 * c13);
  const double B = 4.0 * s13 * c13;
  a.K0 = (R)(1.0 - A - B);
  a.A = (R)A;
  a.B1 = (R)(B * c12);
  a.B2 = (R)(B * s12);
  a.dm21 = th[0];
  a.dm31 = th[1];
  a.dm32 = th[1] - th[0];
  a.n_L = n_L;
  for (int r = 0; r < n_L; ++r) {
    a.KL[r] = kPhase * L[r];
    a.w[r] = (R)(wL ? wL[r] : 1.0 / n_L);
  }
  const int64_t npairs = n >> 1;
  const bool oneL = (n_L == 1 && (!wL || wL[0] == 1.0));
  const bool chunked = sizeof(R) == 8;
  int64_t blocks;
  if (chunked) {
    blocks = std::max<int64_t>(1, (npairs + kPeeChunk - 1) / kPeeChunk);
  } else {
    // 256 groups per CU: enough in flight to keep HBM busy.
    const int64_t want = (npairs + kPeeThreads - 1) / kPeeThreads;
    blocks = std::max<int64_t>(1, std::min(want, (int64_t)cu_count() * 256));
  }
  if (blocks > 0x7fffffffLL) return fail(GNA_E_UNSUPPORTED, "gna_pee: n = %lld too large", (long long)n);
  const dim3 g((unsigned)blocks), t(kPeeThreads);
  if (oneL && chunked)
    hipLaunchKernelGGL((pee_kernel<R, true, true>), g, t, 0, s, E, n, a, (R*)P);
  else if (oneL)
    hipLaunchKernelGGL((pee_kernel<R, true, false>), g, t, 0, s, E, n, a, (R*)P);
  else if (chunked)
    hipLaunchKernelGGL((pee_kernel<R, false, true>), g, t, 0, s, E, n, a, (R*)P);
  else
    hipLaunchKernelGGL((pee_kernel<R, false, false>), g, t, 0, s, E, n, a, (R*)P);
  return check_hip(hipGetLastError(), "gna_pee launch");
}

}  // namespace
}  // namespace gna

extern "C" int gna_pee(const double* E_dev, int64_t n, int32_t n_L, const double* L_km_host,
                       const double* wL_host, const double* theta_host, void* P_dev,
                       int32_t prec, void* stream) {
  using namespace gna;
  clear_error();
  if (n < 0) return fail(GNA_E_INVAL, "gna_pee: n = %lld < 0", (long long)n);
  if (prec != GNA_FP64 && prec != GNA_MIXED) return fail(GNA_E_INVAL, "gna_pee: bad prec %d", prec);
  if (n_L < 1 || n_L > kMaxBaselines)
    return fail(GNA_E_INVAL, "gna_pee: n_L = %d outside 1..%d", n_L, kMaxBaselines);
  if (!L_km_host || !theta_host) return fail(GNA_E_INVAL, "gna_pee: NULL L or theta");
  for (int r = 0; r < n_L; ++r)
    if (!(L_km_host[r] >= 0.0) || !std::isfinite(L_km_host[r]))
      return fail(GNA_E_INVAL, "gna_pee: baseline %d = %g is not a finite value >= 0", r,
                  L_km_host[r]);
  const double s12 = theta_host[2], s13 = theta_host[3];
  if (!(s12 >= 0.0 && s12 <= 1.0 && s13 >= 0.0 && s13 <= 1.0))
    return fail(GNA_E_INVAL, "gna_pee: s12 = %g, s13 = %g must lie in [0, 1]", s12, s13);
  if (!std::isfinite(theta_host[0]) || !std::isfinite(theta_host[1]))
    return fail(GNA_E_INVAL, "gna_pee: dm2 not finite");
  if (n == 0) return GNA_OK;
  if (!E_dev || !P_dev) return fail(GNA_E_INVAL, "gna_pee: NULL device pointer");
  if (((uintptr_t)E_dev & 15) != 0) return fail(GNA_E_INVAL, "gna_pee: E_dev not 16-byte aligned");
  const uintptr_t palign = (prec == GNA_FP64) ? 15 : 7;
  if (((uintptr_t)P_dev & palign) != 0)
    return fail(GNA_E_INVAL, "gna_pee: P_dev not %d-byte aligned", (int)palign + 1);
  hipStream_t s = (hipStream_t)stream;
  if (prec == GNA_FP64)
    return run_pee<double>(E_dev, n, n_L, L_km_host, wL_host, theta_host, P_dev, s);
  return run_pee<float>(E_dev, n, n_L, L_km_host, wL_host, theta_host, P_dev, s);
}

// ---------------------------------------------------------------------------
// Streaming copy (the measured-bandwidth reference for the elementwise kernel
// and the known-size calibration of the memory-traffic counters): 16-byte
// non-temporal loads and stores, two per lane per trip, in the fastest of
// the grid shapes measured on MI355X (512 lanes, 128 groups per CU).
// ---------------------------------------------------------------------------
namespace gna {
namespace {

constexpr int kCopyThreads = 512;

__global__ void __launch_bounds__(kCopyThreads)
    copy_kernel(const double* __restrict__ src, int64_t n, double* __restrict__ dst) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const int64_t npairs = n >> 1;
  const int64_t stride = (int64_t)gridDim.x * kCopyThreads;
  const v2* s2 = reinterpret_cast<const v2*>(src);
  v2* d2 = reinterpret_cast<v2*>(dst);
  int64_t p = (int64_t)blockIdx.x * kCopyThreads + threadIdx.x;
  for (; p + stride < npairs; p += 2 * stride) {
    const v2 a = __builtin_nontemporal_load(s2 + p);
    const v2 b = __builtin_nontemporal_load(s2 + p + stride);
    __builtin_nontemporal_store(a, d2 + p);
    __builtin_nontemporal_store(b, d2 + p + stride);
  }
  if (p < npairs) __builtin_nontemporal_store(__builtin_nontemporal_load(s2 + p), d2 + p);
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) dst[n - 1] = src[n - 1];
}

}  // namespace
}  // namespace gna

extern "C" int gna_stream_copy(const double* src_dev, double* dst_dev, int64_t n, void* stream) {
  using namespace gna;
  clear_error();
  if (n < 0) return fail(GNA_E_INVAL, "gna_stream_copy: n < 0");
  if (n == 0) return GNA_OK;
  if (!src_dev || !dst_dev) return fail(GNA_E_INVAL, "gna_stream_copy: NULL pointer");
  if (((uintptr_t)src_dev | (uintptr_t)dst_dev) & 15)
    return fail(GNA_E_INVAL, "gna_stream_copy: pointers must be 16-byte aligned");
  const int64_t npairs = n >> 1;
  const int64_t want = (npairs + kCopyThreads - 1) / kCopyThreads;
  const int blocks = (int)std::max<int64_t>(1, std::min(want, (int64_t)cu_count() * 128));
  hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(kCopyThreads), 0, (hipStream_t)stream,
                     src_dev, n, dst_dev);
  return check_hip(hipGetLastError(), "gna_stream_copy launch");
}
