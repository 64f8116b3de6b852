// General three-flavour vacuum oscillation probability (Sec. 4.1):
//   P(a -> b) = delta_ab - 4 sum_{i>j} Re(X_ij) sin^2(dm2_ij L / 4E)
//                        + 2 sum_{i>j} Im(X_ij) sin(dm2_ij L / 2E),
//   X_ij = V*_ai V_bi V_aj V*_bj,
// with V the PMNS matrix in the standard parametrisation (three angles, one
// Dirac phase; V -> V* for antineutrinos).  The six coefficients Re/Im X_ij
// depend only on the parameters and are formed on the host per launch; the
// kernel evaluates sin^2 and sin 2phi of the three phases per energy.
#include <algorithm>
#include <cmath>
#include <complex>

#include "gna_internal.h"
#include "gna_math.h"

namespace gna {

// PMNS matrix V[flavour][mass state] = R23 U13(delta) R12.
static void pmns_matrix(double th12, double th13, double th23, double dcp,
                        std::complex<double> V[3][3]) {
  using C = std::complex<double>;
  const double c12 = std::cos(th12), s12 = std::sin(th12);
  const double c13 = std::cos(th13), s13 = std::sin(th13);
  const double c23 = std::cos(th23), s23 = std::sin(th23);
  const C ep = std::polar(1.0, dcp), em = std::polar(1.0, -dcp);
  V[0][0] = C(c12 * c13);
  V[0][1] = C(s12 * c13);
  V[0][2] = s13 * em;
  V[1][0] = -s12 * c23 - c12 * s23 * s13 * ep;
  V[1][1] = c12 * c23 - s12 * s23 * s13 * ep;
  V[1][2] = C(s23 * c13);
  V[2][0] = s12 * s23 - c12 * c23 * s13 * ep;
  V[2][1] = -c12 * s23 - s12 * c23 * s13 * ep;
  V[2][2] = C(c23 * c13);
}

void prob_coefficients(int a, int b, int anti, const double* ang, double* delta, double re[3],
                       double im[3]) {
  std::complex<double> V[3][3];
  pmns_matrix(ang[0], ang[1], ang[2], anti ? -ang[3] : ang[3], V);
  *delta = (a == b) ? 1.0 : 0.0;
  const int pi[3] = {1, 2, 2}, pj[3] = {0, 0, 1};  // pairs i > j: (2,1), (3,1), (3,2)
  for (int t = 0; t < 3; ++t) {
    const int i = pi[t], j = pj[t];
    const std::complex<double> x = std::conj(V[a][i]) * V[b][i] * V[a][j] * std::conj(V[b][j]);
    re[t] = -4.0 * x.real();
    im[t] = 2.0 * x.imag();
  }
}

namespace {

constexpr int kProbThreads = 256;

template <class R>
struct ProbArgs {
  R delta;              // delta_ab
  R re[3], im[3];       // -4 Re X and 2 Im X for the pairs (21, 31, 32)
  double dm[3];         // dm2_21, dm2_31, dm2_32
  int32_t n_L;
  double KL[kMaxBaselines];
  R w[kMaxBaselines];
};

template <class R>
__device__ __forceinline__ R prob_eval(const ProbArgs<R>& a, double E) {
  R acc = R(0);
  for (int r = 0; r < a.n_L; ++r) {
    const double q = (sizeof(R) == 8) ? phase_per_ev2(a.KL[r], E) : phase_per_ev2_fast(a.KL[r], E);
    R p = a.delta;
#pragma unroll
    for (int ij = 0; ij < 3; ++ij) {
      const PhaseTerms<R> t = phase_terms<R>(a.dm[ij] * q);
      p = rfma_t<R>(a.re[ij], t.S, p);
      p = rfma_t<R>(a.im[ij], t.T, p);
    }
    acc = rfma_t<R>(a.w[r], p, acc);
  }
  return acc;
}

template <class R>
__global__ void __launch_bounds__(kProbThreads)
    prob_kernel(const double* __restrict__ E, int64_t n, ProbArgs<R> a, R* __restrict__ P) {
  const int64_t stride = (int64_t)gridDim.x * kProbThreads;
  for (int64_t i = (int64_t)blockIdx.x * kProbThreads + threadIdx.x; i < n; i += stride)
    P[i] = prob_eval<R>(a, __builtin_nontemporal_load(E + i));
}

int g_cus = 0;

template <class R>
int run_prob(const double* E, int64_t n, int a, int b, int nL, const double* L, const double* wL,
             const double* ang, const double* dm, int anti, void* P, hipStream_t s) {
  double delta, re[3], im[3];
  prob_coefficients(a, b, anti, ang, &delta, re, im);
  ProbArgs<R> k{};
  k.delta = (R)delta;
  k.dm[0] = dm[0];
  k.dm[1] = dm[1];
  k.dm[2] = dm[1] - dm[0];
  for (int t = 0; t < 3; ++t) {
    k.re[t] = (R)re[t];
    k.im[t] = (R)im[t];
  }
  k.n_L = nL;
  for (int r = 0; r < nL; ++r) {
    k.KL[r] = kPhase * L[r];
    k.w[r] = (R)(wL ? wL[r] : 1.0 / nL);
  }
  if (g_cus <= 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&g_cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        g_cus <= 0)
      g_cus = 256;
  }
  const int64_t want = (n + kProbThreads - 1) / kProbThreads;
  const int blocks = (int)std::max<int64_t>(1, std::min(want, (int64_t)g_cus * 256));
  hipLaunchKernelGGL(prob_kernel<R>, dim3(blocks), dim3(kProbThreads), 0, s, E, n, k, (R*)P);
  return check_hip(hipGetLastError(), "gna_prob launch");
}

}  // namespace
}  // namespace gna

extern "C" int gna_prob(const double* E_dev, int64_t n, int32_t alpha, int32_t beta, int32_t n_L,
                        const double* L_km_host, const double* wL_host,
                        const double* angles_host, const double* dm2_host, int32_t antineutrino,
                        void* P_dev, int32_t prec, void* stream) {
  using namespace gna;
  clear_error();
  if (n < 0) return fail(GNA_E_INVAL, "gna_prob: n < 0");
  if (alpha < 0 || alpha > 2 || beta < 0 || beta > 2)
    return fail(GNA_E_INVAL, "gna_prob: flavours %d -> %d outside 0..2 (e, mu, tau)", alpha, beta);
  if (prec != GNA_FP64 && prec != GNA_MIXED) return fail(GNA_E_INVAL, "gna_prob: bad prec");
  if (n_L < 1 || n_L > kMaxBaselines) return fail(GNA_E_INVAL, "gna_prob: n_L outside 1..64");
  if (!L_km_host || !angles_host || !dm2_host) return fail(GNA_E_INVAL, "gna_prob: NULL host input");
  for (int r = 0; r < n_L; ++r)
    if (!(L_km_host[r] >= 0.0) || !std::isfinite(L_km_host[r]))
      return fail(GNA_E_INVAL, "gna_prob: baseline %d invalid", r);
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(angles_host[i])) return fail(GNA_E_INVAL, "gna_prob: angle %d not finite", i);
  if (!std::isfinite(dm2_host[0]) || !std::isfinite(dm2_host[1]))
    return fail(GNA_E_INVAL, "gna_prob: dm2 not finite");
  if (n == 0) return GNA_OK;
  if (!E_dev || !P_dev) return fail(GNA_E_INVAL, "gna_prob: NULL device pointer");
  if (((uintptr_t)E_dev & 7) || ((uintptr_t)P_dev & (prec == GNA_FP64 ? 7 : 3)))
    return fail(GNA_E_INVAL, "gna_prob: misaligned device pointer");
  hipStream_t s = (hipStream_t)stream;
  if (prec == GNA_FP64)
    return run_prob<double>(E_dev, n, alpha, beta, n_L, L_km_host, wL_host, angles_host,
                            dm2_host, antineutrino, P_dev, s);
  return run_prob<float>(E_dev, n, alpha, beta, n_L, L_km_host, wL_host, angles_host, dm2_host,
                         antineutrino, P_dev, s);
}
