// FP64 CPU oracle for the reactor-antineutrino prediction chain.
//
// TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
// definition that the GPU library is checked against.  The product library
// never calls, links or includes it: only the test suite, the smoke check and
// the benchmark's CPU-baseline timing load it.  It shares no code, header,
// table or constant generator with the GPU library; the two meet only in the
// seeded input arrays.
//
// Built with  g++ -O2 -fno-fast-math -ffp-contract=off  so every + - * / is a
// single IEEE-754 double rounding in the order written here.  Transcendentals
// are libm's (sin, cos, exp, log, sqrt, erf).
//
// Paper: "CUDA Support in GNA Data Analysis Framework" (arXiv:1804.07682).
// The paper defines only the oscillation probability (Sec. 4.1, the vacuum
// P(nu_alpha -> nu_beta) equation) and the chain structure (Sec. 2.1-2.3,
// Fig. 4: many OscProb instances, one per baseline, sharing one energy
// vector).  Every other step of the chain is a reading, stated where used:
// spectrum, inverse-beta cross section, Gauss-Legendre bin integration,
// Gaussian smearing, Poisson chi^2 and its gradient.
//
// Parameter vector theta = (dm2_21 [eV^2], dm2_31 [eV^2], s12 = sin^2 th12,
// s13 = sin^2 th13, norm).  Energies in MeV, baselines in km.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;

// Phase constant.  The paper writes the phase as dm2_ij L / (4 E) in natural
// units (Sec. 4.1).  With dm2 in eV^2, L in km and E in MeV this is
// K * dm2 * L / E with K = 1e-3 / (4 * hbar*c[eV m]),
// hbar*c = 197.3269804 MeV fm = 1.973269804e-7 eV m, so
// K = 1266.9326794198487 (the decimal literal of that double).
constexpr double K_PHASE = 1266.9326794198487;

constexpr int OK = 0;
constexpr int E_INVAL = -1;
constexpr int E_DOMAIN = -2;

inline double re_part(double x) { return x; }
inline double re_part(const cplx& x) { return x.real(); }

// ---------------------------------------------------------------------------
// Sec. 4.1: general vacuum oscillation probability.
//   P(a->b) = delta_ab - 4 sum_{i>j} Re(V*_ai V_bi V_aj V*_bj) sin^2(dm2_ij L/4E)
//                      + 2 sum_{i>j} Im(V*_ai V_bi V_aj V*_bj) sin(dm2_ij L/2E)
// V is the PMNS matrix in the standard parametrisation by three angles and
// one phase (the paper leaves the parametrisation to the cited textbook).
// ---------------------------------------------------------------------------
void pmns(double th12, double th13, double th23, double dcp, cplx V[3][3]) {
  const double c12 = std::cos(th12), s12 = std::sin(th12);
  const double c13 = std::cos(th13), s13 = std::sin(th13);
  const double c23 = std::cos(th23), s23 = std::sin(th23);
  const cplx eid = std::polar(1.0, dcp);   // e^{+i delta}
  const cplx emid = std::polar(1.0, -dcp); // e^{-i delta}
  V[0][0] = c12 * c13;
  V[0][1] = s12 * c13;
  V[0][2] = s13 * emid;
  V[1][0] = -s12 * c23 - c12 * s23 * s13 * eid;
  V[1][1] = c12 * c23 - s12 * s23 * s13 * eid;
  V[1][2] = s23 * c13;
  V[2][0] = s12 * s23 - c12 * c23 * s13 * eid;
  V[2][1] = -c12 * s23 - s12 * c23 * s13 * eid;
  V[2][2] = c23 * c13;
}

double prob_general(int a, int b, double E, double L, double dm21, double dm31,
                    const cplx V[3][3]) {
  const double dm2[3][3] = {{0.0, -dm21, -dm31},
                            {dm21, 0.0, dm21 - dm31},
                            {dm31, dm31 - dm21, 0.0}};  // dm2[i][j] = m_i^2 - m_j^2
  double p = (a == b) ? 1.0 : 0.0;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < i; ++j) {
      const cplx x = std::conj(V[a][i]) * V[b][i] * V[a][j] * std::conj(V[b][j]);
      const double half_phase = (K_PHASE * L) / E * dm2[i][j];  // dm2 L / 4E
      const double s = std::sin(half_phase);
      p -= 4.0 * x.real() * s * s;
      p += 2.0 * x.imag() * std::sin(2.0 * half_phase);        // dm2 L / 2E
    }
  }
  return p;
}

// Brute force from the amplitude  A(a->b) = sum_i V*_ai V_bi exp(-i m_i^2 L / 2E)
// with m_1^2 = 0; P = |A|^2.  Independent of the sin^2 / Im expansion above.
double prob_amplitude(int a, int b, double E, double L, double dm21, double dm31,
                      const cplx V[3][3]) {
  const double m2[3] = {0.0, dm21, dm31};
  cplx amp(0.0, 0.0);
  for (int i = 0; i < 3; ++i) {
    const double ph = 2.0 * ((K_PHASE * L) / E) * m2[i];  // m_i^2 L / 2E
    amp += std::conj(V[a][i]) * V[b][i] * std::polar(1.0, -ph);
  }
  return std::norm(amp);
}

// ---------------------------------------------------------------------------
// Sec. 4.1 for alpha = beta = e: delta_ee = 1 and the Im term vanishes since
// V*_ei V_ei V_ej V*_ej = |V_ei|^2 |V_ej|^2 is real.  With the mixing given as
// s12 = sin^2 th12, s13 = sin^2 th13:
//   |U_e1|^2 = (1-s12)(1-s13),  |U_e2|^2 = s12 (1-s13),  |U_e3|^2 = s13,
//   P_ee = 1 - 4 (|U_e2 U_e1|^2 sin^2 phi21 + |U_e3 U_e1|^2 sin^2 phi31
//                 + |U_e3 U_e2|^2 sin^2 phi32),
//   phi_ij = dm2_ij * q,  q = (K L) / E,  dm2_32 = dm2_31 - dm2_21.
// Templated on the parameter scalar so that the complex-step check can run
// the very same code with complex parameters.
// ---------------------------------------------------------------------------
template <class T>
T pee_point(double E, double L, const T& dm21, const T& dm31, const T& s12, const T& s13) {
  using std::sin;
  const double q = (K_PHASE * L) / E;
  const T dm32 = dm31 - dm21;
  const T u1 = (1.0 - s12) * (1.0 - s13);
  const T u2 = s12 * (1.0 - s13);
  const T u3 = s13;
  const T sn21 = sin(dm21 * q);
  const T sn31 = sin(dm31 * q);
  const T sn32 = sin(dm32 * q);
  return 1.0 - 4.0 * (u2 * u1 * (sn21 * sn21) + u3 * u1 * (sn31 * sn31) +
                      u3 * u2 * (sn32 * sn32));
}

// Analytic partial derivatives of pee_point with respect to
// (dm2_21, dm2_31, s12, s13), by the product rule on the |U_ei|^2 form:
//   d sin^2(phi)/d phi = sin(2 phi);  d phi21/d dm21 = q, d phi32/d dm21 = -q,
//   d phi31/d dm31 = d phi32/d dm31 = q;
//   d u1/d s12 = -(1-s13), d u2/d s12 = (1-s13);
//   d u1/d s13 = -(1-s12), d u2/d s13 = -s12, d u3/d s13 = 1.
void pee_point_grad(double E, double L, double dm21, double dm31, double s12, double s13,
                    double* p, double dp[4]) {
  const double q = (K_PHASE * L) / E;
  const double dm32 = dm31 - dm21;
  const double u1 = (1.0 - s12) * (1.0 - s13);
  const double u2 = s12 * (1.0 - s13);
  const double u3 = s13;
  const double ph21 = dm21 * q, ph31 = dm31 * q, ph32 = dm32 * q;
  const double S21 = std::sin(ph21) * std::sin(ph21);
  const double S31 = std::sin(ph31) * std::sin(ph31);
  const double S32 = std::sin(ph32) * std::sin(ph32);
  const double T21 = std::sin(2.0 * ph21);
  const double T31 = std::sin(2.0 * ph31);
  const double T32 = std::sin(2.0 * ph32);
  *p = 1.0 - 4.0 * (u2 * u1 * S21 + u3 * u1 * S31 + u3 * u2 * S32);
  // d/d dm21: phi21 and phi32 move.
  dp[0] = -4.0 * (u2 * u1 * T21 * q - u3 * u2 * T32 * q);
  // d/d dm31: phi31 and phi32 move.
  dp[1] = -4.0 * (u3 * u1 * T31 * q + u3 * u2 * T32 * q);
  // d/d s12.
  const double du1_12 = -(1.0 - s13), du2_12 = (1.0 - s13);
  dp[2] = -4.0 * ((du2_12 * u1 + u2 * du1_12) * S21 + u3 * du1_12 * S31 + u3 * du2_12 * S32);
  // d/d s13.
  const double du1_13 = -(1.0 - s12), du2_13 = -s12, du3_13 = 1.0;
  dp[3] = -4.0 * ((du2_13 * u1 + u2 * du1_13) * S21 + (du3_13 * u1 + u3 * du1_13) * S31 +
                  (du3_13 * u2 + u3 * du2_13) * S32);
}

// ---------------------------------------------------------------------------
// Gauss-Legendre rule of order n on [-1, 1] (a reading: the paper names no
// quadrature).  Nodes are the roots of the Legendre polynomial P_n, found by
// Newton's method from the Chebyshev-like start cos(pi (i - 1/4)/(n + 1/2));
// P_n and P_n' come from the three-term recurrence
//   (k+1) P_{k+1}(x) = (2k+1) x P_k(x) - k P_{k-1}(x),
//   P_n'(x) = n (x P_n(x) - P_{n-1}(x)) / (x^2 - 1).
// Weights w_i = 2 / ((1 - x_i^2) P_n'(x_i)^2).  Nodes ascending; the negative
// half mirrors the positive half so the rule is exactly symmetric.
// ---------------------------------------------------------------------------
void legendre(int n, double x, double* pn, double* dpn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { *pn = 1.0; *dpn = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *dpn = n * (x * p1 - p0) / (x * x - 1.0);
}

void gauss_legendre(int n, double* t, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 1; i <= n / 2; ++i) {
    double x = std::cos(pi * (i - 0.25) / (n + 0.5));  // i-th largest root
    for (int it = 0; it < 100; ++it) {
      double pn, dpn;
      legendre(n, x, &pn, &dpn);
      const double dx = pn / dpn;
      x -= dx;
      if (std::fabs(dx) <= 1e-17) break;
    }
    double pn, dpn;
    legendre(n, x, &pn, &dpn);
    const double wi = 2.0 / ((1.0 - x * x) * dpn * dpn);
    t[n - i] = x;   // ascending order: largest root last
    w[n - i] = wi;
    t[i - 1] = -x;
    w[i - 1] = wi;
  }
  if (n % 2 == 1) {
    const int m = n / 2;
    double pn, dpn;
    legendre(n, 0.0, &pn, &dpn);
    t[m] = 0.0;
    w[m] = 2.0 / (dpn * dpn);
  }
}

// ---------------------------------------------------------------------------
// Quadrature points of the bin integration (reading).  Bin j = [e_j, e_{j+1}]
// is cut into n_sub equal sub-intervals with edges
//   u_s = e_j + ((e_{j+1} - e_j) * s) / n_sub  (s < n_sub),  u_{n_sub} = e_{j+1};
// on [a, b] = [u_s, u_{s+1}]:  c = 0.5 (a + b),  h = 0.5 (b - a),
//   E = c + h t_i,  w = h w_i.
// Point index k = (j n_sub + s) order + i.
// ---------------------------------------------------------------------------
void quadrature(int nb, const double* edges, int order, int n_sub, const double* t,
                const double* wt, double* E, double* w) {
  for (int j = 0; j < nb; ++j) {
    const double lo = edges[j], hi = edges[j + 1];
    const double width = hi - lo;
    for (int s = 0; s < n_sub; ++s) {
      const double a = lo + (width * s) / n_sub;
      const double b = (s + 1 == n_sub) ? hi : lo + (width * (s + 1)) / n_sub;
      const double c = 0.5 * (a + b);
      const double h = 0.5 * (b - a);
      for (int i = 0; i < order; ++i) {
        const int64_t k = ((int64_t)j * n_sub + s) * order + i;
        E[k] = c + h * t[i];
        w[k] = h * wt[i];
      }
    }
  }
}

// Reactor spectrum S(E) = exp(a0 + a1 E + a2 E^2 + a3 E^3) (reading: a
// smooth synthetic stand-in, the paper gives no spectrum).
double spectrum(double E, const double a[4]) {
  return std::exp(a[0] + a[1] * E + a[2] * E * E + a[3] * E * E * E);
}

// Inverse-beta-decay cross section up to a constant (reading):
//   sigma(E) = x sqrt(x^2 - m_e^2),  x = E - delta,  and 0 when x <= m_e.
double ibd_xsec(double E, double delta, double me) {
  const double x = E - delta;
  if (x <= me) return 0.0;
  return x * std::sqrt(x * x - me * me);
}

// Gaussian energy-resolution matrix (reading): true energy at the centre of
// bin j, Ebar_j = 0.5 (e_j + e_{j+1}), resolution sigma_j = res_a sqrt(Ebar_j);
// R_ij is the probability to reconstruct in bin i:
//   R_ij = 0.5 [erf((e_{i+1} - Ebar_j)/(sqrt2 sigma_j)) - erf((e_i - Ebar_j)/(sqrt2 sigma_j))].
// Dense, row-major R[i * nb + j].  No column renormalisation.
void smearing_matrix(int nb, const double* edges, double res_a, double* R) {
  const double sqrt2 = std::sqrt(2.0);
  for (int j = 0; j < nb; ++j) {
    const double ebar = 0.5 * (edges[j] + edges[j + 1]);
    const double sig = res_a * std::sqrt(ebar);
    const double den = sqrt2 * sig;
    for (int i = 0; i < nb; ++i) {
      R[(int64_t)i * nb + j] =
          0.5 * (std::erf((edges[i + 1] - ebar) / den) - std::erf((edges[i] - ebar) / den));
    }
  }
}

// Poisson chi^2 in the Baker-Cousins form (reading: the paper names no
// statistic):  chi2 = 2 sum_i [nu_i - d_i + d_i ln(d_i / nu_i)],
// with d ln(d/nu) = 0 at d = 0.  Returns E_DOMAIN if some nu_i <= 0.
template <class T>
int chi2_of(int nb, const T* nu, const double* d, T* out) {
  using std::log;
  T acc = 0.0;
  for (int i = 0; i < nb; ++i) {
    if (!(re_part(nu[i]) > 0.0)) return E_DOMAIN;
    T term = nu[i] - d[i];
    if (d[i] > 0.0) term = term + d[i] * log(d[i] / nu[i]);
    acc = acc + term;
  }
  *out = 2.0 * acc;
  return OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

typedef struct {
  int32_t n_bins;
  const double* edges;  // n_bins + 1, strictly increasing
  int32_t gl_order;     // >= 1
  int32_t n_sub;        // >= 1
  int32_t n_L;
  const double* L_km;   // n_L
  const double* wL;     // n_L, or NULL for 1/n_L
  double spec[4];       // spectrum exponent coefficients a0..a3
  double xsec_delta;    // 1.293 MeV
  double m_e;           // 0.511 MeV
  double n0;            // overall normalisation N0
  double res_a;         // sigma_E = res_a sqrt(E)
  const double* data;   // n_bins observed counts (>= 0)
} oracle_chain_desc;

double oracle_phase_constant(void) { return K_PHASE; }

int oracle_prob_general(int32_t alpha, int32_t beta, int64_t n, const double* E, double L,
                        double dm21, double dm31, double th12, double th13, double th23,
                        double dcp, double* P) {
  if (alpha < 0 || alpha > 2 || beta < 0 || beta > 2 || n < 0) return E_INVAL;
  cplx V[3][3];
  pmns(th12, th13, th23, dcp, V);
  for (int64_t i = 0; i < n; ++i) P[i] = prob_general(alpha, beta, E[i], L, dm21, dm31, V);
  return OK;
}

int oracle_prob_amplitude(int32_t alpha, int32_t beta, int64_t n, const double* E, double L,
                          double dm21, double dm31, double th12, double th13, double th23,
                          double dcp, double* P) {
  if (alpha < 0 || alpha > 2 || beta < 0 || beta > 2 || n < 0) return E_INVAL;
  cplx V[3][3];
  pmns(th12, th13, th23, dcp, V);
  for (int64_t i = 0; i < n; ++i) P[i] = prob_amplitude(alpha, beta, E[i], L, dm21, dm31, V);
  return OK;
}

// Baseline-weighted survival probability Pbar(E) = sum_r wL_r P_ee(E; L_r)
// (Fig. 4: one OscProb per baseline on a shared energy vector; reading: the
// weights are caller-given, 1/n_L when wL is NULL).
// theta = (dm21, dm31, s12, s13).  Optional dP[n][4] = d Pbar / d theta.
int oracle_pee(int64_t n, const double* E, int32_t n_L, const double* L, const double* wL,
               const double* theta, double* P, double* dP, int32_t n_threads) {
  if (n < 0 || n_L < 1 || !theta || (n > 0 && (!E || !P)) || !L) return E_INVAL;
#ifdef _OPENMP
  const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0, dacc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < n_L; ++r) {
      const double wr = wL ? wL[r] : 1.0 / n_L;
      if (dP) {
        double p, dp[4];
        pee_point_grad(E[i], L[r], theta[0], theta[1], theta[2], theta[3], &p, dp);
        acc += wr * p;
        for (int c = 0; c < 4; ++c) dacc[c] += wr * dp[c];
      } else {
        acc += wr * pee_point<double>(E[i], L[r], theta[0], theta[1], theta[2], theta[3]);
      }
    }
    P[i] = acc;
    if (dP)
      for (int c = 0; c < 4; ++c) dP[i * 4 + c] = dacc[c];
  }
  (void)n_threads;
  return OK;
}

int oracle_gauss_legendre(int32_t n, double* t, double* w) {
  if (n < 1 || n > 256 || !t || !w) return E_INVAL;
  gauss_legendre(n, t, w);
  return OK;
}

int oracle_quadrature(int32_t nb, const double* edges, int32_t order, int32_t n_sub, double* E,
                      double* w) {
  if (nb < 1 || order < 1 || order > 256 || n_sub < 1 || !edges || !E || !w) return E_INVAL;
  std::vector<double> t(order), wt(order);
  gauss_legendre(order, t.data(), wt.data());
  quadrature(nb, edges, order, n_sub, t.data(), wt.data(), E, w);
  return OK;
}

// f_k = N0 w_k S(E_k) sigma(E_k): the parameter-independent flux x cross
// section x quadrature weight of every point.
int oracle_flux_xsec(int64_t n, const double* E, const double* w, const double* spec4,
                     double xsec_delta, double m_e, double n0, double* f) {
  if (n < 0 || !spec4) return E_INVAL;
  for (int64_t k = 0; k < n; ++k)
    f[k] = n0 * w[k] * spectrum(E[k], spec4) * ibd_xsec(E[k], xsec_delta, m_e);
  return OK;
}

int oracle_smearing(int32_t nb, const double* edges, double res_a, double* R) {
  if (nb < 1 || !edges || !R || !(res_a >= 0.0)) return E_INVAL;
  smearing_matrix(nb, edges, res_a, R);
  return OK;
}

namespace {

struct Tables {
  int nb = 0, npts = 0, ppb = 0;
  std::vector<double> E, w, f, R;
};

int build_tables(const oracle_chain_desc* d, Tables* tb) {
  if (!d || d->n_bins < 1 || !d->edges || d->gl_order < 1 || d->gl_order > 256 ||
      d->n_sub < 1 || d->n_L < 1 || !d->L_km || !d->data)
    return E_INVAL;
  for (int j = 0; j < d->n_bins; ++j)
    if (!(d->edges[j + 1] > d->edges[j])) return E_INVAL;
  tb->nb = d->n_bins;
  tb->ppb = d->gl_order * d->n_sub;
  tb->npts = tb->nb * tb->ppb;
  tb->E.resize(tb->npts);
  tb->w.resize(tb->npts);
  tb->f.resize(tb->npts);
  tb->R.resize((size_t)tb->nb * tb->nb);
  std::vector<double> t(d->gl_order), wt(d->gl_order);
  gauss_legendre(d->gl_order, t.data(), wt.data());
  quadrature(tb->nb, d->edges, d->gl_order, d->n_sub, t.data(), wt.data(), tb->E.data(),
             tb->w.data());
  for (int k = 0; k < tb->npts; ++k)
    tb->f[k] = d->n0 * tb->w[k] * spectrum(tb->E[k], d->spec) *
               ibd_xsec(tb->E[k], d->xsec_delta, d->m_e);
  smearing_matrix(tb->nb, d->edges, d->res_a, tb->R.data());
  return OK;
}

// One parameter point of the chain:
//   Pbar_k = sum_r wL_r P_ee(E_k; L_r)
//   mu_j   = norm sum_{k in bin j} f_k Pbar_k                 (bin integration)
//   nu_i   = sum_j R_ij mu_j                                  (smearing)
//   chi2   = Baker-Cousins chi^2(nu, d)
// and, when grad != NULL, the gradient by the chain rule:
//   J_jc = norm sum_k f_k d Pbar_k / d theta_c,  mu0_j = sum_k f_k Pbar_k,
//   gnu_i = d chi2 / d nu_i = 2 (1 - d_i / nu_i),
//   gmu_j = sum_i R_ij gnu_i,
//   d chi2 / d theta_c = sum_j gmu_j J_jc,   d chi2 / d norm = sum_j gmu_j mu0_j.
int eval_point(const oracle_chain_desc* d, const Tables& tb, const double* th, double* chi2,
               double* grad, double* mu_out, double* nu_out) {
  const int nb = tb.nb, ppb = tb.ppb;
  std::vector<double> mu0(nb, 0.0), J((size_t)nb * 4, 0.0), nu(nb, 0.0);
  for (int j = 0; j < nb; ++j) {
    double acc = 0.0, dacc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < ppb; ++i) {
      const int k = j * ppb + i;
      double pbar = 0.0, dpbar[4] = {0.0, 0.0, 0.0, 0.0};
      for (int r = 0; r < d->n_L; ++r) {
        const double wr = d->wL ? d->wL[r] : 1.0 / d->n_L;
        double p, dp[4];
        pee_point_grad(tb.E[k], d->L_km[r], th[0], th[1], th[2], th[3], &p, dp);
        pbar += wr * p;
        for (int c = 0; c < 4; ++c) dpbar[c] += wr * dp[c];
      }
      acc += tb.f[k] * pbar;
      for (int c = 0; c < 4; ++c) dacc[c] += tb.f[k] * dpbar[c];
    }
    mu0[j] = acc;
    for (int c = 0; c < 4; ++c) J[(size_t)j * 4 + c] = th[4] * dacc[c];
  }
  for (int i = 0; i < nb; ++i) {
    double acc = 0.0;
    for (int j = 0; j < nb; ++j) acc += tb.R[(size_t)i * nb + j] * (th[4] * mu0[j]);
    nu[i] = acc;
  }
  const int rc = chi2_of<double>(nb, nu.data(), d->data, chi2);
  if (mu_out)
    for (int j = 0; j < nb; ++j) mu_out[j] = th[4] * mu0[j];
  if (nu_out)
    for (int i = 0; i < nb; ++i) nu_out[i] = nu[i];
  if (rc != OK) return rc;
  if (grad) {
    std::vector<double> gnu(nb), gmu(nb, 0.0);
    for (int i = 0; i < nb; ++i) gnu[i] = 2.0 * (1.0 - d->data[i] / nu[i]);
    for (int j = 0; j < nb; ++j) {
      double acc = 0.0;
      for (int i = 0; i < nb; ++i) acc += tb.R[(size_t)i * nb + j] * gnu[i];
      gmu[j] = acc;
    }
    for (int c = 0; c < 5; ++c) grad[c] = 0.0;
    for (int j = 0; j < nb; ++j) {
      for (int c = 0; c < 4; ++c) grad[c] += gmu[j] * J[(size_t)j * 4 + c];
      grad[4] += gmu[j] * mu0[j];
    }
  }
  return OK;
}

// The same chain with complex parameters (no gradient): used only for the
// complex-step derivative d chi2/d theta_c = Im chi2(theta + i h e_c) / h.
int eval_point_complex(const oracle_chain_desc* d, const Tables& tb, const cplx* th, cplx* chi2) {
  const int nb = tb.nb, ppb = tb.ppb;
  std::vector<cplx> mu(nb), nu(nb);
  for (int j = 0; j < nb; ++j) {
    cplx acc = 0.0;
    for (int i = 0; i < ppb; ++i) {
      const int k = j * ppb + i;
      cplx pbar = 0.0;
      for (int r = 0; r < d->n_L; ++r) {
        const double wr = d->wL ? d->wL[r] : 1.0 / d->n_L;
        pbar += wr * pee_point<cplx>(tb.E[k], d->L_km[r], th[0], th[1], th[2], th[3]);
      }
      acc += tb.f[k] * pbar;
    }
    mu[j] = th[4] * acc;
  }
  for (int i = 0; i < nb; ++i) {
    cplx acc = 0.0;
    for (int j = 0; j < nb; ++j) acc += tb.R[(size_t)i * nb + j] * mu[j];
    nu[i] = acc;
  }
  return chi2_of<cplx>(nb, nu.data(), d->data, chi2);
}

}  // namespace

// Chain for B parameter points sharing one geometry.  params[B][5];
// chi2[B]; grad[B][5], mu[B][nb], nu[B][nb] optional (NULL).
// Returns the first nonzero per-point status (E_DOMAIN when some nu <= 0).
int oracle_chain(const oracle_chain_desc* d, int32_t B, const double* params, double* chi2,
                 double* grad, double* mu, double* nu, int32_t n_threads) {
  if (B < 0 || (B > 0 && (!params || !chi2))) return E_INVAL;
  Tables tb;
  int rc = build_tables(d, &tb);
  if (rc != OK) return rc;
  for (int b = 0; b < B; ++b) {
    const double* th = params + 5 * b;
    if (!(th[2] >= 0.0 && th[2] <= 1.0 && th[3] >= 0.0 && th[3] <= 1.0)) return E_DOMAIN;
  }
  int status = OK;
#ifdef _OPENMP
  const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic) num_threads(nt)
#endif
  for (int b = 0; b < B; ++b) {
    const int r = eval_point(d, tb, params + 5 * b, chi2 + b, grad ? grad + 5 * b : nullptr,
                             mu ? mu + (size_t)b * tb.nb : nullptr,
                             nu ? nu + (size_t)b * tb.nb : nullptr);
    if (r != OK) {
#ifdef _OPENMP
#pragma omp critical
#endif
      if (status == OK) status = r;
    }
  }
  (void)n_threads;
  return status;
}

// Independent fits, each with its own geometry and one parameter point:
// descs[n_fits], params[n_fits][5], chi2[n_fits], grad[n_fits][5] (optional).
int oracle_fitset(int32_t n_fits, const oracle_chain_desc* descs, const double* params,
                  double* chi2, double* grad, int32_t n_threads) {
  if (n_fits < 0 || (n_fits > 0 && (!descs || !params || !chi2))) return E_INVAL;
  int status = OK;
#ifdef _OPENMP
  const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic) num_threads(nt)
#endif
  for (int f = 0; f < n_fits; ++f) {
    Tables tb;
    int r = build_tables(descs + f, &tb);
    if (r == OK)
      r = eval_point(descs + f, tb, params + 5 * f, chi2 + f, grad ? grad + 5 * f : nullptr,
                     nullptr, nullptr);
    if (r != OK) {
#ifdef _OPENMP
#pragma omp critical
#endif
      if (status == OK) status = r;
    }
  }
  (void)n_threads;
  return status;
}

// Complex-step derivative of chi2 with respect to each of the 5 parameters:
// dchi2[c] = Im chi2(theta + i h e_c) / h  (exact to rounding for analytic
// chains; no subtractive cancellation, so h may be tiny, e.g. 1e-30 |theta_c|).
int oracle_chi2_complex_step(const oracle_chain_desc* d, const double* params, const double* h,
                             double* dchi2) {
  if (!params || !h || !dchi2) return E_INVAL;
  Tables tb;
  int rc = build_tables(d, &tb);
  if (rc != OK) return rc;
  for (int c = 0; c < 5; ++c) {
    cplx th[5];
    for (int i = 0; i < 5; ++i) th[i] = cplx(params[i], 0.0);
    th[c] = cplx(params[c], h[c]);
    cplx chi2;
    rc = eval_point_complex(d, tb, th, &chi2);
    if (rc != OK) return rc;
    dchi2[c] = chi2.imag() / h[c];
  }
  return OK;
}

// ---------------------------------------------------------------------------
// The chain's steps as separate vector-in / vector-out transformations
// (Sec. 2.1, Fig. 2: each transformation maps input vectors to an output
// vector), over n_vec vectors stored one after another.
// ---------------------------------------------------------------------------

// Bin integration: mu[v][j] = sum_{i < ppb} w[j ppb + i] x[v][j ppb + i]
// (w NULL: every weight 1), the terms added in ascending i.
int oracle_bin_integrate(int64_t n_vec, int32_t nb, int32_t ppb, const double* x,
                         const double* w, double* mu) {
  if (n_vec < 0 || nb < 1 || ppb < 1 || (n_vec > 0 && (!x || !mu))) return E_INVAL;
  const int64_t npts = (int64_t)nb * ppb;
  for (int64_t v = 0; v < n_vec; ++v)
    for (int j = 0; j < nb; ++j) {
      double acc = 0.0;
      for (int i = 0; i < ppb; ++i) {
        const int64_t k = (int64_t)j * ppb + i;
        acc += (w ? w[k] : 1.0) * x[v * npts + k];
      }
      mu[v * nb + j] = acc;
    }
  return OK;
}

// Smearing with a dense row-major R[n_rows][n_cols]:
//   transpose = 0:  y[v][i] = sum_j R_ij x[v][j]   (x: n_cols, y: n_rows)
//   transpose = 1:  y[v][j] = sum_i R_ij x[v][i]   (x: n_rows, y: n_cols)
// the second being the adjoint step of the gradient (gmu = R^T gnu).
int oracle_smear_apply(int32_t n_rows, int32_t n_cols, const double* R, int32_t transpose,
                       int64_t n_vec, const double* x, double* y) {
  if (n_rows < 1 || n_cols < 1 || !R || n_vec < 0 || (transpose != 0 && transpose != 1) ||
      (n_vec > 0 && (!x || !y)))
    return E_INVAL;
  const int n_in = transpose ? n_rows : n_cols, n_out = transpose ? n_cols : n_rows;
  for (int64_t v = 0; v < n_vec; ++v)
    for (int o = 0; o < n_out; ++o) {
      double acc = 0.0;
      for (int c = 0; c < n_in; ++c) {
        const double r = transpose ? R[(int64_t)c * n_cols + o] : R[(int64_t)o * n_cols + c];
        acc += r * x[v * n_in + c];
      }
      y[v * n_out + o] = acc;
    }
  return OK;
}

// Baker-Cousins chi^2 of n_vec predictions nu[v][nb] against data
// d + v d_stride (d_stride 0: one data vector for all), and optionally its
// derivative d chi2 / d nu_i = 2 (1 - d_i / nu_i) into dchi2_dnu[v][nb].
// Returns E_DOMAIN (outputs of that vector unset) if some nu_i <= 0.
int oracle_chi2(int32_t nb, int64_t n_vec, const double* nu, const double* d, int64_t d_stride,
                double* chi2, double* dchi2_dnu) {
  if (nb < 1 || n_vec < 0 || d_stride < 0 || (n_vec > 0 && (!nu || !d || !chi2))) return E_INVAL;
  int status = OK;
  for (int64_t v = 0; v < n_vec; ++v) {
    const double* nv = nu + v * nb;
    const double* dv = d + v * d_stride;
    const int rc = chi2_of<double>(nb, nv, dv, chi2 + v);
    if (rc != OK) {
      if (status == OK) status = rc;
      continue;
    }
    if (dchi2_dnu)
      for (int i = 0; i < nb; ++i) dchi2_dnu[v * nb + i] = 2.0 * (1.0 - dv[i] / nv[i]);
  }
  return status;
}

// Complex-step derivative of the chi^2 above with respect to each nu_i:
// out[i] = Im chi2(nu + i h_i e_i) / h_i (pins the closed form 2 (1 - d/nu)
// without using it).
int oracle_chi2_dnu_complex_step(int32_t nb, const double* nu, const double* d, const double* h,
                                 double* out) {
  if (nb < 1 || !nu || !d || !h || !out) return E_INVAL;
  std::vector<cplx> z(nb);
  for (int i = 0; i < nb; ++i) {
    for (int k = 0; k < nb; ++k) z[k] = cplx(nu[k], 0.0);
    z[i] = cplx(nu[i], h[i]);
    cplx c;
    const int rc = chi2_of<cplx>(nb, z.data(), d, &c);
    if (rc != OK) return rc;
    out[i] = c.imag() / h[i];
  }
  return OK;
}

}  // extern "C"
