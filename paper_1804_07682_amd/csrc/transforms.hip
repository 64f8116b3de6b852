// The chain's steps as separate vector-in / vector-out transformations
// (Sec. 2.1, Fig. 2: a transformation maps read-only input vectors to an
// output vector it owns), each over a batch of vectors in FP64:
//   gna_bin_integrate  mu[v][j] = sum_i w[j ppb + i] x[v][j ppb + i]
//   gna_smear          y = R x or y = R^T x (the adjoint step of the gradient)
//   gna_chi2           Baker-Cousins chi^2 and d chi^2 / d nu
// Reading any of these intermediate results costs one launch and one output
// (Sec. 4.2, Fig. 6); the fused chain kernels are the fast path for the whole
// chain.  Every sum runs in a fixed order, so results do not depend on
// scheduling.
#include <algorithm>
#include <cmath>

#include "gna_internal.h"
#include "gna_math.h"

namespace gna {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxGridY = 65535;

// ---------------------------------------------------------------------------
// Bin integration: G lanes per bin (a power of two), each lane summing the
// bin's points i = lane, lane + G, ...; the G partial sums are then folded by
// butterfly shuffles.  Bins of one work-group are consecutive, so a wavefront
// reads a contiguous run of points.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
    bin_integrate_kernel(const double* __restrict__ x, const double* __restrict__ w,
                         int64_t n_vec, int nb, int ppb, int G, double* __restrict__ mu) {
  const int per_group = kThreads / G;
  const int j = blockIdx.x * per_group + (int)threadIdx.x / G;
  const int lane = (int)threadIdx.x & (G - 1);
  const int64_t npts = (int64_t)nb * ppb;
  for (int64_t v = blockIdx.y; v < n_vec; v += gridDim.y) {
    double acc = 0.0;
    if (j < nb) {
      const int64_t base = (int64_t)j * ppb;
      const double* xv = x + v * npts + base;
      if (w) {
        for (int i = lane; i < ppb; i += G) acc = dfma(w[base + i], xv[i], acc);
      } else {
        for (int i = lane; i < ppb; i += G) acc += xv[i];
      }
    }
    // every lane of the wavefront takes part in the shuffles
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if (j < nb && lane == 0) mu[v * nb + j] = acc;
  }
}

// ---------------------------------------------------------------------------
// Smearing: y[v][o] = sum_c A(o, c) x[v][c], with A(o, c) = R[o][c] (R x) or
// R[c][o] (R^T x).  A work-group owns 64 outputs of 4 vectors (one output per
// lane); the contraction runs over 64-wide tiles of A, staged through LDS as
// T[c][o] so that the lanes of a wavefront read consecutive words, with the
// matching slice of the 4 vectors beside it.  Global loads are coalesced in
// both modes: along c (R x, where T is written transposed) or along o (R^T x).
// Each output adds its terms in ascending c.
// ---------------------------------------------------------------------------
constexpr int kTileO = 64;
constexpr int kTileC = 64;
constexpr int kVecPerGroup = kThreads / kTileO;  // 4

template <bool TRANSPOSE>
__global__ void __launch_bounds__(kThreads)
    smear_tiled_kernel(const double* __restrict__ R, int n_rows, int n_cols,
                       const double* __restrict__ x, int64_t n_vec, double* __restrict__ y) {
  __shared__ double T[kTileC][kTileO + 1];
  __shared__ double xs[kVecPerGroup][kTileC];
  const int n_in = TRANSPOSE ? n_rows : n_cols;
  const int n_out = TRANSPOSE ? n_cols : n_rows;
  const int t = threadIdx.x;
  const int ol = t & (kTileO - 1);
  const int vq = t / kTileO;
  const int o0 = blockIdx.x * kTileO;
  for (int64_t v0 = (int64_t)blockIdx.y * kVecPerGroup; v0 < n_vec;
       v0 += (int64_t)gridDim.y * kVecPerGroup) {
    const int64_t v = v0 + vq;
    double acc = 0.0;
    for (int c0 = 0; c0 < n_in; c0 += kTileC) {
      for (int e = t; e < kTileC * kTileO; e += kThreads) {
        int cl, oo;
        if (TRANSPOSE) {  // consecutive lanes: consecutive o of row c of R
          cl = e / kTileO;
          oo = e & (kTileO - 1);
        } else {          // consecutive lanes: consecutive c of row o of R
          oo = e / kTileC;
          cl = e & (kTileC - 1);
        }
        const int c = c0 + cl, o = o0 + oo;
        double a = 0.0;
        if (c < n_in && o < n_out)
          a = TRANSPOSE ? R[(int64_t)c * n_cols + o] : R[(int64_t)o * n_cols + c];
        T[cl][oo] = a;
      }
      {
        const int cl = t & (kTileC - 1);
        const int c = c0 + cl;
        xs[vq][cl] = (v < n_vec && c < n_in) ? x[v * n_in + c] : 0.0;
      }
      __syncthreads();
      const int nc = min(kTileC, n_in - c0);
      for (int cl = 0; cl < nc; ++cl) acc = dfma(T[cl][ol], xs[vq][cl], acc);
      __syncthreads();
    }
    const int o = o0 + ol;
    if (v < n_vec && o < n_out) y[v * n_out + o] = acc;
  }
}

// ---------------------------------------------------------------------------
// chi^2 = 2 sum_i [nu_i - d_i + d_i ln(d_i / nu_i)] (d ln(d/nu) = 0 at d = 0)
// and d chi^2 / d nu_i = 2 (1 - d_i / nu_i): one work-group per vector, lanes
// take bins i = tid, tid + 256, ..., then a fixed-order tree through LDS.  A
// bin with nu <= 0 (or NaN) makes that vector's chi^2 NaN, and its derivative
// entry NaN.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads)
    chi2_batch_kernel(const double* __restrict__ nu, const double* __restrict__ d,
                      int64_t d_stride, int nb, int64_t n_vec, double* __restrict__ chi2,
                      double* __restrict__ dnu) {
  __shared__ double part[kThreads];
  __shared__ int bad_any;
  for (int64_t v = blockIdx.x; v < n_vec; v += gridDim.x) {
    const double* nv = nu + v * nb;
    const double* dv = d + v * d_stride;
    if (threadIdx.x == 0) bad_any = 0;
    __syncthreads();
    double s = 0.0;
    bool bad = false;
    for (int i = threadIdx.x; i < nb; i += kThreads) {
      const double n = nv[i], di = dv[i];
      const double q = quot_pos(di, n);  // NaN for n <= 0 or NaN
      bad |= !(n > 0.0);
      double term = n - di;
      if (di > 0.0) term = dfma(di, log_pos(q), term);
      s += term;
      if (dnu) dnu[v * nb + i] = 2.0 * (1.0 - q);
    }
    if (bad) bad_any = 1;  // benign race: every writer stores 1
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) chi2[v] = bad_any ? __builtin_nan("") : 2.0 * part[0];
    __syncthreads();  // part and bad_any are reused by the next vector
  }
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7) == 0; }

}  // namespace
}  // namespace gna

using namespace gna;

extern "C" int gna_bin_integrate(const double* x_dev, const double* w_dev, int64_t n_vec,
                                 int32_t n_bins, int32_t ppb, double* mu_dev, void* stream) {
  clear_error();
  if (n_vec < 0) return fail(GNA_E_INVAL, "gna_bin_integrate: n_vec = %lld < 0", (long long)n_vec);
  if (n_bins < 1 || ppb < 1)
    return fail(GNA_E_INVAL, "gna_bin_integrate: n_bins = %d, ppb = %d must be >= 1", n_bins, ppb);
  if ((int64_t)n_bins * ppb > (1LL << 40))
    return fail(GNA_E_INVAL, "gna_bin_integrate: n_bins * ppb too large");
  if (n_vec == 0) return GNA_OK;
  if (!x_dev || !mu_dev) return fail(GNA_E_INVAL, "gna_bin_integrate: NULL device pointer");
  if (!aligned8(x_dev) || !aligned8(w_dev) || !aligned8(mu_dev))
    return fail(GNA_E_INVAL, "gna_bin_integrate: pointers must be 8-byte aligned");
  int G = 1;
  while (G < kWave && 2 * G <= ppb) G *= 2;
  const int per_group = kThreads / G;
  const unsigned gx = (unsigned)((n_bins + per_group - 1) / per_group);
  const unsigned gy = (unsigned)std::min<int64_t>(n_vec, kMaxGridY);
  hipLaunchKernelGGL(bin_integrate_kernel, dim3(gx, gy), dim3(kThreads), 0, (hipStream_t)stream,
                     x_dev, w_dev, n_vec, (int)n_bins, (int)ppb, G, mu_dev);
  return check_hip(hipGetLastError(), "gna_bin_integrate launch");
}

extern "C" int gna_smear(const double* R_dev, int32_t n_rows, int32_t n_cols, int32_t transpose,
                         const double* x_dev, int64_t n_vec, double* y_dev, void* stream) {
  clear_error();
  if (n_rows < 1 || n_cols < 1)
    return fail(GNA_E_INVAL, "gna_smear: R is %d x %d", n_rows, n_cols);
  if (transpose != 0 && transpose != 1)
    return fail(GNA_E_INVAL, "gna_smear: transpose = %d not 0/1", transpose);
  if (n_vec < 0) return fail(GNA_E_INVAL, "gna_smear: n_vec = %lld < 0", (long long)n_vec);
  if (n_vec == 0) return GNA_OK;
  if (!R_dev || !x_dev || !y_dev) return fail(GNA_E_INVAL, "gna_smear: NULL device pointer");
  if (!aligned8(R_dev) || !aligned8(x_dev) || !aligned8(y_dev))
    return fail(GNA_E_INVAL, "gna_smear: pointers must be 8-byte aligned");
  const int n_out = transpose ? n_cols : n_rows;
  const unsigned gx = (unsigned)((n_out + kTileO - 1) / kTileO);
  const int64_t groups = (n_vec + kVecPerGroup - 1) / kVecPerGroup;
  const unsigned gy = (unsigned)std::min<int64_t>(groups, kMaxGridY);
  hipStream_t s = (hipStream_t)stream;
  if (transpose)
    hipLaunchKernelGGL(smear_tiled_kernel<true>, dim3(gx, gy), dim3(kThreads), 0, s, R_dev,
                       (int)n_rows, (int)n_cols, x_dev, n_vec, y_dev);
  else
    hipLaunchKernelGGL(smear_tiled_kernel<false>, dim3(gx, gy), dim3(kThreads), 0, s, R_dev,
                       (int)n_rows, (int)n_cols, x_dev, n_vec, y_dev);
  return check_hip(hipGetLastError(), "gna_smear launch");
}

extern "C" int gna_chi2(const double* nu_dev, const double* data_dev, int64_t data_stride,
                        int32_t n_bins, int64_t n_vec, double* chi2_dev, double* dchi2_dnu_dev,
                        void* stream) {
  clear_error();
  if (n_bins < 1) return fail(GNA_E_INVAL, "gna_chi2: n_bins = %d < 1", n_bins);
  if (n_vec < 0) return fail(GNA_E_INVAL, "gna_chi2: n_vec = %lld < 0", (long long)n_vec);
  if (data_stride != 0 && data_stride != n_bins)
    return fail(GNA_E_INVAL, "gna_chi2: data_stride = %lld must be 0 or n_bins",
                (long long)data_stride);
  if (n_vec == 0) return GNA_OK;
  if (!nu_dev || !data_dev || !chi2_dev) return fail(GNA_E_INVAL, "gna_chi2: NULL device pointer");
  if (!aligned8(nu_dev) || !aligned8(data_dev) || !aligned8(chi2_dev) || !aligned8(dchi2_dnu_dev))
    return fail(GNA_E_INVAL, "gna_chi2: pointers must be 8-byte aligned");
  const unsigned g = (unsigned)std::min<int64_t>(n_vec, 1 << 20);
  hipLaunchKernelGGL(chi2_batch_kernel, dim3(g), dim3(kThreads), 0, (hipStream_t)stream, nu_dev,
                     data_dev, data_stride, (int)n_bins, n_vec, chi2_dev, dchi2_dnu_dev);
  return check_hip(hipGetLastError(), "gna_chi2 launch");
}
