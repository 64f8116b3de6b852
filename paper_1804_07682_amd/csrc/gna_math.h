// Device math of the oscillation step: phase, reduction modulo pi/2 and the
// trigonometric terms of the survival probability (Sec. 4.1).
//
// The library is compiled with -ffp-contract=off: every fused multiply-add
// below is written out, every other operation is a single IEEE rounding.
#pragma once

#include <hip/hip_runtime.h>

#include "trig_coeffs.h"

namespace gna {

// Phase constant: the Sec. 4.1 phase dm2_ij L / (4 E) (natural units) equals
// K * dm2[eV^2] * L[km] / E[MeV] with K = 1e-3 / (4 hbar c[eV m]),
// hbar c = 197.3269804 MeV fm; K is the double 1266.9326794198487.
constexpr double kPhase = 1266.9326794198487;

__device__ __forceinline__ double dfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float ffma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// phi = m * pi/2 + r with |r| <= pi/4 (+ rounding), m = nearest integer to
// phi * 2/pi.  t = phi * 2/pi + 1.5 * 2^52 is rounded once by the FMA to an
// integer held in the low mantissa bits, so m = t - 1.5 * 2^52 exactly and the
// parity of m is bit 0 of t (valid for |phi| < 2^50).  Two-part Cody-Waite
// subtraction with FMAs: each step rounds an exactly formed product once; the
// dropped third part of pi/2 contributes |m| * 1.5e-33, far below an ulp of r.
// tlo: the low word of t (bit 0 = parity of m).
__device__ __forceinline__ double reduce_pio2_t(double phi, int& tlo) {
  const double magic = 6755399441055744.0;  // 1.5 * 2^52
  const double t = dfma(phi, GNA_TWO_OVER_PI, magic);
  const double m = t - magic;
  tlo = __double2loint(t);
  double r = dfma(-m, GNA_PIO2_1, phi);
  r = dfma(-m, GNA_PIO2_2, r);
  return r;
}

__device__ __forceinline__ double reduce_pio2(double phi, bool& odd) {
  int tlo;
  const double r = reduce_pio2_t(phi, tlo);
  odd = (tlo & 1) != 0;
  return r;
}

// Reciprocal of E > 0 to ~1 ulp.  The seed rsq(E)^2 is NaN for E < 0 and
// inf for E = 0 (which the first Newton step turns into NaN), so a
// non-positive energy yields NaN without a separate test; two Newton steps
// take the ~2^-25 seed to full precision.
__device__ __forceinline__ double recip_pos(double E) {
  double y = __builtin_amdgcn_rsq(E);
  y = y * y;
  y = dfma(y, dfma(-E, y, 1.0), y);
  y = dfma(y, dfma(-E, y, 1.0), y);
  return y;
}

// q = KL / E rounded to nearest: quotient from the reciprocal, then one
// Markstein correction with the exactly computed remainder KL - E q.  For
// normal-range operands (energies and baselines here) this is the correctly
// rounded quotient, so FP64 phases match (K L) / E evaluated by an IEEE
// division; non-positive E gives NaN.
__device__ __forceinline__ double phase_per_ev2(double KL, double E) {
  const double y = recip_pos(E);
  const double q = KL * y;
  return dfma(dfma(-E, q, KL), y, q);
}

// a / b for b > 0, rounded to nearest in the normal range (the same
// reciprocal-and-correction steps as the phase quotient above); NaN for b <= 0
// or NaN.  Shorter dependent chain than the IEEE division sequence.
__device__ __forceinline__ double quot_pos(double a, double b) { return phase_per_ev2(a, b); }

// q = KL / E within ~2 ulp (mixed precision: the phase needs ~1e-13 relative).
__device__ __forceinline__ double phase_per_ev2_fast(double KL, double E) {
  return KL * recip_pos(E);
}

// Natural logarithm in FP64 for the chi^2 tail: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), f = m - 1 (exact), s = f / (2 + f) from a refined
// reciprocal, ln(1 + f) = 2 atanh(s) = 2 s (1 + s^2/3 + s^4/5 + ... + s^20/21)
// (s^2 <= 0.0295, so the dropped terms are below 1e-18 relative), plus e ln 2
// in two parts.  Within 2 ulp for every positive finite x, subnormals
// included; 0 gives -inf, +inf gives +inf, negative or NaN x gives NaN.
__device__ __forceinline__ double log_pos(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  if (m < 0.70710678118654752440) {
    m = m + m;
    e -= 1;
  }
  const double f = m - 1.0;
  const double den = 2.0 + f;
  double r = __builtin_amdgcn_rcp(den);
  r = dfma(r, dfma(-den, r, 1.0), r);
  r = dfma(r, dfma(-den, r, 1.0), r);
  double s = f * r;
  s = dfma(dfma(-den, s, f), r, s);
  const double z = s * s;
  double p = 1.0 / 21;
  p = dfma(p, z, 1.0 / 19);
  p = dfma(p, z, 1.0 / 17);
  p = dfma(p, z, 1.0 / 15);
  p = dfma(p, z, 1.0 / 13);
  p = dfma(p, z, 1.0 / 11);
  p = dfma(p, z, 1.0 / 9);
  p = dfma(p, z, 1.0 / 7);
  p = dfma(p, z, 1.0 / 5);
  p = dfma(p, z, 1.0 / 3);
  const double l1 = dfma((s + s) * z, p, s + s);
  const double de = (double)e;
  const double lx = dfma(de, 0x1.62e42fefa3800p-1, dfma(de, 0x1.ef35793c76730p-45, l1));
  if (x > 0.0 && x < __builtin_huge_val()) return lx;
  return x == 0.0 ? -__builtin_huge_val() : (x > 0.0 ? x : __builtin_nan(""));
}

// Natural logarithm with a table of 257 entries (a table-driven reduction):
// x = m 2^e with m in [sqrt(1/2), sqrt(2)); k = floor(362 m - 255.5) in
// [0, 256] picks c_k = (k + 256) / 362 (c_106 = 1 exactly); tab[2k] = r_k, the
// double nearest 1 / c_k, and tab[2k+1] = -ln r_k to the nearest double (both
// computed once on the host); f = m r_k - 1 is rounded once (|f| <= 0.002) and
//   ln x = e ln 2 + (-ln r_k) + log1p(f),  log1p(f) = f - f^2/2 + ... - f^6/6,
// the dropped terms below 2e-20.  Within a few ulp; near x = 1, k = 106 and
// r_k = 1, so nothing cancels.  Same special cases as log_pos (the index is
// clamped so that they read the table in bounds).
constexpr int kLogTab = 257;

__device__ __forceinline__ double log_tab(double x, const double* tab) {
  double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  if (m < 0.70710678118654752440) {
    m = m + m;
    e -= 1;
  }
  int k = (int)dfma(m, 362.0, -255.5);
  k = k < 0 ? 0 : (k > kLogTab - 1 ? kLogTab - 1 : k);
  const double r = tab[2 * k], mlr = tab[2 * k + 1];
  const double f = dfma(m, r, -1.0);
  double p = dfma(f, -1.0 / 6, 0.2);
  p = dfma(f, p, -0.25);
  p = dfma(f, p, 1.0 / 3);
  p = dfma(f, p, -0.5);
  const double l1 = dfma(f * f, p, f);
  const double de = (double)e;
  const double lx = dfma(de, 0x1.62e42fefa3800p-1, dfma(de, 0x1.ef35793c76730p-45, mlr + l1));
  if (x > 0.0 && x < __builtin_huge_val()) return lx;
  return x == 0.0 ? -__builtin_huge_val() : (x > 0.0 ? x : __builtin_nan(""));
}

// sin r, cos r on |r| <= pi/4 (minimax kernels from trig_coeffs.h).
__device__ __forceinline__ void sincos_kernel(double r, double& s, double& c) {
  const double x = r * r;
  double ps = GNA_SD5;
  ps = dfma(ps, x, GNA_SD4);
  ps = dfma(ps, x, GNA_SD3);
  ps = dfma(ps, x, GNA_SD2);
  ps = dfma(ps, x, GNA_SD1);
  ps = dfma(ps, x, GNA_SD0);
  s = dfma(r * x, ps, r);
  double pc = GNA_CD5;
  pc = dfma(pc, x, GNA_CD4);
  pc = dfma(pc, x, GNA_CD3);
  pc = dfma(pc, x, GNA_CD2);
  pc = dfma(pc, x, GNA_CD1);
  pc = dfma(pc, x, GNA_CD0);
  c = dfma(x * x, pc, dfma(-0.5, x, 1.0));
}

__device__ __forceinline__ void sincos_kernel(float r, float& s, float& c) {
  const float x = r * r;
  float ps = GNA_SF2;
  ps = ffma(ps, x, GNA_SF1);
  ps = ffma(ps, x, GNA_SF0);
  s = ffma(r * x, ps, r);
  float pc = GNA_CF2;
  pc = ffma(pc, x, GNA_CF1);
  pc = ffma(pc, x, GNA_CF0);
  c = ffma(x * x, pc, ffma(-0.5f, x, 1.0f));
}

// sin^2 r on |r| <= pi/4.
__device__ __forceinline__ double sin2_kernel(double r) {
  const double x = r * r;
  double p = GNA_QD6;
  p = dfma(p, x, GNA_QD5);
  p = dfma(p, x, GNA_QD4);
  p = dfma(p, x, GNA_QD3);
  p = dfma(p, x, GNA_QD2);
  p = dfma(p, x, GNA_QD1);
  p = dfma(p, x, GNA_QD0);
  return dfma(x * x, p, x);
}

// sin^2 r on |r| <= pi/4 with one coefficient fewer (relative error 3.2e-14):
// the FP64 elementwise kernel, bound by memory bandwidth and by its vector
// instruction count, where the result is held to 1e-12.
__device__ __forceinline__ double sin2_kernel_short(double r) {
  const double x = r * r;
  double p = GNA_QS5;
  p = dfma(p, x, GNA_QS4);
  p = dfma(p, x, GNA_QS3);
  p = dfma(p, x, GNA_QS2);
  p = dfma(p, x, GNA_QS1);
  p = dfma(p, x, GNA_QS0);
  return dfma(x * x, p, x);
}

__device__ __forceinline__ float sin2_kernel(float r) {
  const float x = r * r;
  float p = GNA_QF3;
  p = ffma(p, x, GNA_QF2);
  p = ffma(p, x, GNA_QF1);
  p = ffma(p, x, GNA_QF0);
  return ffma(x * x, p, x);
}

template <class R>
__device__ __forceinline__ R to_r(double x) { return static_cast<R>(x); }

__device__ __forceinline__ double rfma_t_impl(double a, double b, double c) { return dfma(a, b, c); }
__device__ __forceinline__ float rfma_t_impl(float a, float b, float c) { return ffma(a, b, c); }
template <class R>
__device__ __forceinline__ R rfma_t(R a, R b, R c) { return rfma_t_impl(a, b, c); }

// cos^2(phi) only (probability without tangents).  The reduction is FP64;
// the kernel runs in R (double, or float for the mixed-precision mode).
template <class R>
__device__ __forceinline__ R cos2_phase(double phi) {
  bool odd;
  const double r = reduce_pio2(phi, odd);
  const R s2 = sin2_kernel(to_r<R>(r));
  const R c2 = R(1) - s2;  // >= 1/2: no cancellation
  return odd ? s2 : c2;
}

// sin^2(phi), cos^2(phi) and sin(2 phi) of one phase.
template <class R>
struct PhaseTerms {
  R S, C, T;
};

template <class R>
__device__ __forceinline__ PhaseTerms<R> phase_terms(double phi) {
  if constexpr (sizeof(R) == 8) {
    // FP64 without selects: with h = 1/2 - sin^2 r and sigma = (-1)^m,
    // sin^2 phi = 1/2 - sigma h, cos^2 phi = 1/2 + sigma h and
    // sin 2phi = sigma sin 2r; sigma enters as the sign bit (bit 0 of the
    // reduction's t, shifted to bit 63).  C - S = 2 sigma h exactly; S and
    // C are within 2^-54 absolute of their correctly rounded values.
    int tlo;
    const double r = reduce_pio2_t(phi, tlo);
    double s, c;
    sincos_kernel(r, s, c);
    const unsigned long long sg = (unsigned long long)(unsigned)tlo << 63;
    const double h = __longlong_as_double(
        (long long)((unsigned long long)__double_as_longlong(0.5 - s * s) ^ sg));
    const double t = 2.0 * (s * c);
    PhaseTerms<R> out;
    out.S = 0.5 - h;
    out.C = 0.5 + h;
    out.T = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(t) ^ sg));
    return out;
  } else {
    bool odd;
    const double r = reduce_pio2(phi, odd);
    R s, c;
    sincos_kernel(to_r<R>(r), s, c);
    const R s2 = s * s, c2 = c * c;
    const R sc = s * c;
    PhaseTerms<R> out;
    out.S = odd ? c2 : s2;                 // sin^2(m pi/2 + r)
    out.C = odd ? s2 : c2;                 // cos^2(m pi/2 + r)
    out.T = odd ? R(-2) * sc : R(2) * sc;  // sin(m pi + 2 r) = (-1)^m sin 2r
    return out;
  }
}

// Terms of phi32 = phi31 - phi21 from those of phi21 and phi31 by the
// angle-difference formulas for the doubled angles (cos 2phi = C - S,
// sin 2phi = T):
//   cos 2phi32 = (C31 - S31)(C21 - S21) + T31 T21,
//   sin 2phi32 = T31 (C21 - S21) - (C31 - S31) T21,
//   S32 = (1 - cos 2phi32) / 2,   C32 = (1 + cos 2phi32) / 2.
// A third reduction and polynomial pair is replaced by a few products; the
// implied phase is phi31 - phi21 of the two rounded phases, which differs
// from (dm2_31 - dm2_21) q by a few ulps of phi31: harmless in mixed
// precision, but at 1300 km it moves FP64 gradients by ~1e-12 relative, so
// FP64 corrects it (phase_terms_diff64 below).
template <class R>
__device__ __forceinline__ PhaseTerms<R> phase_terms_diff(const PhaseTerms<R>& t21,
                                                          const PhaseTerms<R>& t31) {
  const R u21 = t21.C - t21.S, u31 = t31.C - t31.S;
  const R c2 = rfma_t<R>(u31, u21, t31.T * t21.T);
  PhaseTerms<R> out;
  out.T = rfma_t<R>(t31.T, u21, -(u31 * t21.T));
  out.S = rfma_t<R>(R(-0.5), c2, R(0.5));
  out.C = rfma_t<R>(R(0.5), c2, R(0.5));
  return out;
}

// Per-parameter-point coefficients of P_ee written in the all-positive form
//   P = K0 + A cos^2 phi21 + B1 cos^2 phi31 + B2 cos^2 phi32,
//   A = 4 s12 (1-s12) (1-s13)^2, B = 4 s13 (1-s13), B1 = B (1-s12), B2 = B s12,
//   K0 = 1 - A - B,
// which equals the Sec. 4.1 expression 1 - A sin^2 phi21 - B1 sin^2 phi31 -
// B2 sin^2 phi32 (cos^2 = 1 - sin^2) and keeps every term non-negative.
// Derivatives (sin 2phi = d sin^2 phi / d phi; phi_ij = dm2_ij q):
//   dP/d dm21 = q (-A T21 + B2 T32)
//   dP/d dm31 = -q (B1 T31 + B2 T32)
//   dP/d s12  = -dA12 S21 - B (S32 - S31),   dA12 = 4 (1 - 2 s12) (1-s13)^2
//   dP/d s13  = -dA13 S21 - dB13 ((1-s12) S31 + s12 S32),
//               dA13 = -8 s12 (1-s12) (1-s13),  dB13 = 4 (1 - 2 s13)
template <class R>
struct PeeCoef {
  double dm21, dm31, dm32;
  double dm32e;  // (dm2_31 - dm2_21) - dm32, the exact error of the subtraction
  R K0, A, B, B1, B2, s12, c12, dA12, dA13, dB13;
  bool bad;
};

template <class R>
__device__ __forceinline__ PeeCoef<R> pee_coef(const double* th) {
  PeeCoef<R> k;
  k.dm21 = th[0];
  k.dm31 = th[1];
  k.dm32 = th[1] - th[0];
  {  // two-sum: the subtraction's rounding error, exactly
    const double a = th[1], b = -th[0];
    const double bb = k.dm32 - a;
    k.dm32e = (a - (k.dm32 - bb)) + (b - bb);
  }
  const double s12 = th[2], s13 = th[3];
  k.bad = !(s12 >= 0.0 && s12 <= 1.0 && s13 >= 0.0 && s13 <= 1.0);
  const double c13 = 1.0 - s13, c12 = 1.0 - s12;
  const double A = 4.0 * s12 * c12 * (c13 * c13);
  const double B = 4.0 * s13 * c13;
  k.K0 = to_r<R>(1.0 - A - B);
  k.A = to_r<R>(A);
  k.B = to_r<R>(B);
  k.B1 = to_r<R>(B * c12);
  k.B2 = to_r<R>(B * s12);
  k.s12 = to_r<R>(s12);
  k.c12 = to_r<R>(c12);
  k.dA12 = to_r<R>(4.0 * (1.0 - 2.0 * s12) * (c13 * c13));
  k.dA13 = to_r<R>(-8.0 * s12 * c12 * c13);
  k.dB13 = to_r<R>(4.0 * (1.0 - 2.0 * s13));
  return k;
}

// FP64 terms of phi32 = RN(dm32 q) from those of phi21 and phi31.  The
// doubled-angle formulas of phase_terms_diff give the terms of theta =
// phi31 - phi21 of the two rounded phases, which differs from phi32 by
//   Delta = phi32 - theta = -e q + (r31 - r21) - r32,
// with r_ij = dm2_ij q - phi_ij the exact residuals of the three products (by
// FMA) and e the exact error of dm32 = dm2_31 - dm2_21; every term is below
// ~1e-12 rad, so rotating the doubled angle by 2 Delta to first order,
//   cos 2phi32 = cos 2theta - 2 Delta sin 2theta,
//   sin 2phi32 = sin 2theta + 2 Delta cos 2theta,
// leaves an error near 1e-24: the terms are those of the oracle's phi32 to a
// few ulps, for about half the work of a third reduction and polynomial pair.
template <class R>
__device__ __forceinline__ PhaseTerms<double> phase_terms_diff64(const PhaseTerms<double>& t21,
                                                                 const PhaseTerms<double>& t31,
                                                                 double q, const PeeCoef<R>& k) {
  const double p21 = k.dm21 * q, p31 = k.dm31 * q, p32 = k.dm32 * q;
  const double r21 = dfma(k.dm21, q, -p21), r31 = dfma(k.dm31, q, -p31);
  const double r32 = dfma(k.dm32, q, -p32);
  const double d2 = 2.0 * dfma(-k.dm32e, q, (r31 - r21) - r32);
  const double u21 = t21.C - t21.S, u31 = t31.C - t31.S;
  const double c2 = dfma(u31, u21, t31.T * t21.T);
  const double s2 = dfma(t31.T, u21, -(u31 * t21.T));
  const double c2r = dfma(-d2, s2, c2);
  PhaseTerms<double> out;
  out.T = dfma(d2, c2, s2);
  out.S = dfma(-0.5, c2r, 0.5);
  out.C = dfma(0.5, c2r, 0.5);
  return out;
}

// P_ee and its four parameter derivatives at phase-per-eV^2 q, with the
// trigonometric terms of phase i (0: phi21, 1: phi31) given by terms(i) and
// those of phi32 derived from the two (phase_terms_diff, and in FP64 with the
// correction to RN(dm32 q) of phase_terms_diff64).  Each phase's terms are
// folded into P and the tangents as soon as they are available, which keeps
// few values live at once.
template <class R, bool GRAD, class Terms>
__device__ __forceinline__ void pee_accumulate(const PeeCoef<R>& k, R qr, Terms terms, R& P,
                                               R dP[4]) {
  const PhaseTerms<R> t21 = terms(0);
  R p = rfma_t<R>(k.A, t21.C, k.K0);
  R d0 = R(0), d1 = R(0), d2 = R(0), d3 = R(0);
  if (GRAD) {
    d0 = -(k.A * t21.T);
    d2 = -(k.dA12 * t21.S);
    d3 = -(k.dA13 * t21.S);
  }
  const PhaseTerms<R> t31 = terms(1);
  p = rfma_t<R>(k.B1, t31.C, p);
  if (GRAD) {
    d1 = -(k.B1 * t31.T);
    d2 = rfma_t<R>(k.B, t31.S, d2);
    d3 = d3 - k.dB13 * (k.c12 * t31.S);
  }
  PhaseTerms<R> t32;
  if constexpr (sizeof(R) == 8)
    t32 = phase_terms_diff64<R>(t21, t31, (double)qr, k);
  else
    t32 = phase_terms_diff<R>(t21, t31);
  P = rfma_t<R>(k.B2, t32.C, p);
  if (GRAD) {
    const R bt = k.B2 * t32.T;
    dP[0] = qr * (d0 + bt);
    dP[1] = qr * (d1 - bt);
    dP[2] = d2 - k.B * t32.S;
    dP[3] = d3 - k.dB13 * (k.s12 * t32.S);
  }
}

// P_ee and its four parameter derivatives at phase-per-eV^2 q = (K L) / E.
template <class R, bool GRAD>
__device__ __forceinline__ void pee_point(const PeeCoef<R>& k, double q, R& P, R dP[4]) {
  pee_accumulate<R, GRAD>(
      k, to_r<R>(q),
      [&](int i) { return phase_terms<R>((i == 0 ? k.dm21 : k.dm31) * q); },
      P, dP);
}

}  // namespace gna
