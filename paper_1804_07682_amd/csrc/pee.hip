// Elementwise survival probability over a resident energy vector (Sec. 4.1):
// P[i] = sum_r w_r P_ee(E[i]; L_r, theta).
//
// HBM-streaming kernel: 16-byte non-temporal loads of two energies per lane
// and 16-byte (FP64) or 8-byte (mixed) stores, software-pipelined; the probability needs only
// cos^2 of each phase, so one sin^2 polynomial per phase is evaluated
// (cos^2 = 1 - sin^2 >= 1/2 on the reduced argument).  Phases and their
// reduction are FP64 in both modes; q = KL / E comes from a refined
// reciprocal (~2 ulp), see pee_eval.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "gna_internal.h"
#include "gna_math.h"

namespace gna {

void pee_coefficients(double s12, double s13, double* K0, double* A, double* B1, double* B2) {
  const double c12 = 1.0 - s12, c13 = 1.0 - s13;
  const double a = 4.0 * s12 * c12 * (c13 * c13);
  const double b = 4.0 * s13 * c13;
  *K0 = 1.0 - a - b;
  *A = a;
  *B1 = b * c12;
  *B2 = b * s12;
}

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

// cos^2 phi in FP64 with the short sin^2 kernel (see pee_eval), without a
// select: with h = 1/2 - sin^2 r, cos^2 phi = 1/2 + h for even m and
// 1/2 - h (= sin^2 r) for odd m, so the parity (bit 0 of the reduction's t)
// goes into the sign bit of h by one exclusive or.  Each form is within an
// ulp and a half of the selected one (1/2 - sin^2 r is exact for sin^2 r >=
// 1/4, and otherwise rounds at most 2^-54 absolute).
__device__ __forceinline__ double cos2_phase_short(double phi) {
  int tlo;
  const double r = reduce_pio2_t(phi, tlo);
  const double h = 0.5 - sin2_kernel_short(r);
  const unsigned long long hb = (unsigned long long)__double_as_longlong(h) ^
                                ((unsigned long long)(unsigned)tlo << 63);
  return __longlong_as_double((long long)hb) + 0.5;
}

template <class R>
__device__ __forceinline__ R cos2_stream(double phi) {
  if constexpr (sizeof(R) == 8)
    return cos2_phase_short(phi);
  else
    return cos2_phase<R>(phi);
}

// In both modes q = (K L) * (1/E) comes from the refined reciprocal without
// the quotient's correction step (within 2 ulp), and FP64 takes the short
// sin^2 kernel: this kernel streams from HBM and its time is set by its
// vector instruction count as much as by memory, and the two approximations
// together move P by at most a few 1e-13 relative (at 1300 km, where phases
// reach 2e3 rad), inside the 1e-12 FP64 target.  The fused chain kernels
// keep the correctly rounded phase and the full polynomials.
template <class R, bool ONE_L>
__device__ __forceinline__ R pee_eval(const PeeArgs<R>& a, double E) {
  R acc = R(0);
  const int nL = ONE_L ? 1 : a.n_L;
  for (int r = 0; r < nL; ++r) {
    const double q = phase_per_ev2_fast(a.KL[r], E);
    const R c21 = cos2_stream<R>(a.dm21 * q);
    const R c31 = cos2_stream<R>(a.dm31 * q);
    const R c32 = cos2_stream<R>(a.dm32 * q);
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
  double K0, A, B1, B2;
  pee_coefficients(th[2], th[3], &K0, &A, &B1, &B2);
  a.K0 = (R)K0;
  a.A = (R)A;
  a.B1 = (R)B1;
  a.B2 = (R)B2;
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

namespace gna {
namespace {

// Host-side checks shared by the resident and the host-memory entry points.
int check_pee_args(const char* who, int64_t n, int32_t n_L, const double* L, const double* th,
                   int32_t prec) {
  if (n < 0) return fail(GNA_E_INVAL, "%s: n = %lld < 0", who, (long long)n);
  if (prec != GNA_FP64 && prec != GNA_MIXED) return fail(GNA_E_INVAL, "%s: bad prec %d", who, prec);
  if (n_L < 1 || n_L > kMaxBaselines)
    return fail(GNA_E_INVAL, "%s: n_L = %d outside 1..%d", who, n_L, kMaxBaselines);
  if (!L || !th) return fail(GNA_E_INVAL, "%s: NULL L or theta", who);
  for (int r = 0; r < n_L; ++r)
    if (!(L[r] >= 0.0) || !std::isfinite(L[r]))
      return fail(GNA_E_INVAL, "%s: baseline %d = %g is not a finite value >= 0", who, r, L[r]);
  const double s12 = th[2], s13 = th[3];
  if (!(s12 >= 0.0 && s12 <= 1.0 && s13 >= 0.0 && s13 <= 1.0))
    return fail(GNA_E_INVAL, "%s: s12 = %g, s13 = %g must lie in [0, 1]", who, s12, s13);
  if (!std::isfinite(th[0]) || !std::isfinite(th[1]))
    return fail(GNA_E_INVAL, "%s: dm2 not finite", who);
  return GNA_OK;
}

int launch_pee(const double* E, int64_t n, int32_t n_L, const double* L, const double* wL,
               const double* th, void* P, int32_t prec, hipStream_t s) {
  if (prec == GNA_FP64) return run_pee<double>(E, n, n_L, L, wL, th, P, s);
  return run_pee<float>(E, n, n_L, L, wL, th, P, s);
}

// Streams and an event of the transfer pipeline, per device, created at the
// first call on that device and kept until the process ends.
constexpr int kMaxDevices = 64;
struct PipeDev {
  bool ready = false;
  hipStream_t st[GNA_PIPE_MAX_STREAMS];
  hipEvent_t start;
  unsigned char* scratch = nullptr;  // this device's copy of `scratch` below
};
PipeDev g_pipe[kMaxDevices];
std::mutex g_pipe_mu;   // guards g_pipe
std::mutex g_pipe_run;  // one pipelined call at a time (they share streams and the event)

// Staging buffers of gna_pee_host_noalloc: a file-scope device array, so that
// entry point needs no workspace.  Every device that loads the library holds
// its own copy until the process ends; host code reaches a device's copy only
// through the address hipGetSymbolAddress returns with that device current.
constexpr size_t kNoallocScratchBytes = (size_t)GNA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

// Library resources of the current device: the pipeline streams and event,
// and the device address of `scratch`.  Idempotent.
int pipe_resources(PipeDev*& out) {
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= kMaxDevices) return fail(GNA_E_UNSUPPORTED, "device %d", dev);
  std::lock_guard<std::mutex> lock(g_pipe_mu);
  PipeDev& d = g_pipe[dev];
  if (!d.ready) {
    void* addr = nullptr;
    if ((rc = check_hip(hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)),
                        "hipGetSymbolAddress (no-allocation scratch)")))
      return rc;
    if (!addr || ((uintptr_t)addr & 255) != 0)
      return fail(GNA_E_HIP, "no-allocation scratch at %p is not 256-byte aligned", addr);
    for (int k = 0; k < GNA_PIPE_MAX_STREAMS; ++k)
      if ((rc = check_hip(hipStreamCreateWithFlags(&d.st[k], hipStreamNonBlocking),
                          "hipStreamCreateWithFlags")))
        return rc;
    if ((rc = check_hip(hipEventCreateWithFlags(&d.start, hipEventDisableTiming),
                        "hipEventCreateWithFlags")))
      return rc;
    d.scratch = (unsigned char*)addr;
    d.ready = true;
  }
  out = &d;
  return GNA_OK;
}

size_t pipe_slot_bytes(int64_t chunk, int32_t prec) {
  const size_t osz = prec == GNA_FP64 ? 8 : 4;
  return align_up((size_t)chunk * 8, 256) + align_up((size_t)chunk * osz, 256);
}

// Host-side checks of the pipelined entry points; *need receives the staging
// bytes (n_streams slots of chunk energies and chunk results).
int check_pipe_args(const char* who, int64_t chunk, int32_t n_streams, int32_t prec,
                    size_t* need) {
  if (chunk < 2 || (chunk & 1))
    return fail(GNA_E_INVAL, "%s: chunk = %lld must be even and >= 2", who, (long long)chunk);
  if (n_streams < 1 || n_streams > GNA_PIPE_MAX_STREAMS)
    return fail(GNA_E_INVAL, "%s: n_streams = %d outside 1..%d", who, n_streams,
                GNA_PIPE_MAX_STREAMS);
  if (prec != GNA_FP64 && prec != GNA_MIXED) return fail(GNA_E_INVAL, "%s: bad prec %d", who, prec);
  *need = (size_t)n_streams * pipe_slot_bytes(chunk, prec);
  return GNA_OK;
}

// The pipeline itself, on staging memory ws (device, 256-byte aligned, at
// least n_streams slots).  ws == nullptr: this device's `scratch`.
int pee_host_run(const double* E_host, int64_t n, int32_t n_L, const double* L_km_host,
                 const double* wL_host, const double* theta_host, void* P_host, int32_t prec,
                 unsigned char* ws, int64_t chunk, int32_t n_streams, void* stream) {
  std::lock_guard<std::mutex> running(g_pipe_run);
  PipeDev* pd = nullptr;
  int rc = pipe_resources(pd);
  if (rc) return rc;
  if (!ws) ws = pd->scratch;
  // Start after the work already queued on the caller's stream.
  if ((rc = check_hip(hipEventRecord(pd->start, (hipStream_t)stream), "hipEventRecord")))
    return rc;
  for (int k = 0; k < n_streams; ++k)
    if ((rc = check_hip(hipStreamWaitEvent(pd->st[k], pd->start, 0), "hipStreamWaitEvent")))
      return rc;
  const size_t osz = prec == GNA_FP64 ? 8 : 4;
  const size_t slot = pipe_slot_bytes(chunk, prec);
  // Chunk i on stream i % n_streams: a slot's buffers are reused only after
  // the same (in-order) stream has copied its previous chunk back.
  for (int64_t i = 0, off = 0; off < n; ++i, off += chunk) {
    const int k = (int)(i % n_streams);
    const int64_t m = std::min(chunk, n - off);
    double* E_dev = (double*)(ws + k * slot);
    void* P_dev = ws + k * slot + align_up((size_t)chunk * 8, 256);
    hipStream_t s = pd->st[k];
    if ((rc = check_hip(hipMemcpyAsync(E_dev, E_host + off, (size_t)m * 8, hipMemcpyHostToDevice, s),
                        "hipMemcpyAsync (energies)")))
      break;
    if ((rc = launch_pee(E_dev, m, n_L, L_km_host, wL_host, theta_host, P_dev, prec, s))) break;
    if ((rc = check_hip(hipMemcpyAsync((unsigned char*)P_host + (size_t)off * osz, P_dev,
                                       (size_t)m * osz, hipMemcpyDeviceToHost, s),
                        "hipMemcpyAsync (probabilities)")))
      break;
  }
  // Drain every stream (also after an error, so no copy is left in flight).
  for (int k = 0; k < n_streams; ++k) {
    const int r2 = check_hip(hipStreamSynchronize(pd->st[k]), "hipStreamSynchronize");
    if (!rc) rc = r2;
  }
  return rc;
}

}  // namespace
}  // namespace gna

extern "C" int gna_pee(const double* E_dev, int64_t n, int32_t n_L, const double* L_km_host,
                       const double* wL_host, const double* theta_host, void* P_dev,
                       int32_t prec, void* stream) {
  using namespace gna;
  clear_error();
  int rc = check_pee_args("gna_pee", n, n_L, L_km_host, theta_host, prec);
  if (rc) return rc;
  if (n == 0) return GNA_OK;
  if (!E_dev || !P_dev) return fail(GNA_E_INVAL, "gna_pee: NULL device pointer");
  if (((uintptr_t)E_dev & 15) != 0) return fail(GNA_E_INVAL, "gna_pee: E_dev not 16-byte aligned");
  const uintptr_t palign = (prec == GNA_FP64) ? 15 : 7;
  if (((uintptr_t)P_dev & palign) != 0)
    return fail(GNA_E_INVAL, "gna_pee: P_dev not %d-byte aligned", (int)palign + 1);
  return launch_pee(E_dev, n, n_L, L_km_host, wL_host, theta_host, P_dev, prec,
                    (hipStream_t)stream);
}

extern "C" int gna_pee_host_workspace_size(int64_t chunk, int32_t n_streams, int32_t prec,
                                           size_t* bytes) {
  using namespace gna;
  clear_error();
  if (!bytes) return fail(GNA_E_INVAL, "gna_pee_host_workspace_size: NULL bytes");
  return check_pipe_args("gna_pee_host_workspace_size", chunk, n_streams, prec, bytes);
}

extern "C" int gna_pee_host(const double* E_host, int64_t n, int32_t n_L, const double* L_km_host,
                            const double* wL_host, const double* theta_host, void* P_host,
                            int32_t prec, void* workspace_dev, size_t workspace_bytes,
                            int64_t chunk, int32_t n_streams, void* stream) {
  using namespace gna;
  clear_error();
  int rc = check_pee_args("gna_pee_host", n, n_L, L_km_host, theta_host, prec);
  if (rc) return rc;
  size_t need = 0;
  if ((rc = check_pipe_args("gna_pee_host", chunk, n_streams, prec, &need))) return rc;
  if (n == 0) return GNA_OK;
  if (!E_host || !P_host) return fail(GNA_E_INVAL, "gna_pee_host: NULL host pointer");
  if (!workspace_dev || ((uintptr_t)workspace_dev & 255) != 0)
    return fail(GNA_E_INVAL, "gna_pee_host: workspace NULL or not 256-byte aligned");
  if (workspace_bytes < need)
    return fail(GNA_E_WORKSPACE, "gna_pee_host: workspace %zu bytes, needs %zu", workspace_bytes,
                need);
  return pee_host_run(E_host, n, n_L, L_km_host, wL_host, theta_host, P_host, prec,
                      (unsigned char*)workspace_dev, chunk, n_streams, stream);
}

extern "C" int gna_pee_host_noalloc(const double* E_host, int64_t n, int32_t n_L,
                                    const double* L_km_host, const double* wL_host,
                                    const double* theta_host, void* P_host, int32_t prec,
                                    int64_t chunk, int32_t n_streams, void* stream) {
  using namespace gna;
  clear_error();
  int rc = check_pee_args("gna_pee_host_noalloc", n, n_L, L_km_host, theta_host, prec);
  if (rc) return rc;
  size_t need = 0;
  if ((rc = check_pipe_args("gna_pee_host_noalloc", chunk, n_streams, prec, &need))) return rc;
  if (need > kNoallocScratchBytes)
    return fail(GNA_E_INVAL,
                "gna_pee_host_noalloc: %d streams of %lld-element chunks need %zu staging bytes, "
                "the static scratch holds %zu",
                n_streams, (long long)chunk, need, kNoallocScratchBytes);
  if (n == 0) return GNA_OK;
  if (!E_host || !P_host) return fail(GNA_E_INVAL, "gna_pee_host_noalloc: NULL host pointer");
  return pee_host_run(E_host, n, n_L, L_km_host, wL_host, theta_host, P_host, prec, nullptr,
                      chunk, n_streams, stream);
}

extern "C" int gna_device_init(void) {
  using namespace gna;
  clear_error();
  PipeDev* pd = nullptr;
  return pipe_resources(pd);
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
