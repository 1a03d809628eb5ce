// Per-query accuracy certificate of the float32-operand exact KDE (device
// side, shared by the forward reductions and the adjoint's); see cert.hip.
#pragma once

#include "common.h"
#include "kernels.h"

namespace deann {

namespace cert_detail {

constexpr double kU = 5.9604644775390625e-08;   // 2^-24, unit roundoff of float32
constexpr double kLn2 = 0.6931471805599453;
constexpr double kLog = 18.0;                   // ln(2 / delta), delta = 3e-8 per query

// Bernstein's inequality for a sum of independent zero-mean terms of variance
// sum V and single terms at most b: |sum| <= t with probability 1 - delta.
__device__ inline double bernstein(double V, double b) {
  const double c = b * kLog / 3.0;
  return c + sqrt(c * c + 2.0 * V * kLog);
}

// True when query i must be re-evaluated.  T: the sweep's kernel sum (before
// the Gaussian query factor f, which scales T and sqrt(A) alike), A: sum of
// K^2, y2: for the Gaussian kernel the sum of K times its exponent (-log2 K,
// before f), for the exponential kernel the largest K; yn = ||y~||^2.  AN >= 0:
// the sum over pairs of (K N)^2 with the pair's own N = ||x~||^2 + ||y~||^2
// (Gaussian: in units of L = Lf, the float32 log2-scaled 1/(2h^2)), which
// replaces the largest row norm in the variance of the dot-product roundings;
// AN < 0: not available.  AK >= 0 (three-part bfloat16 operands): the sum over
// pairs of K N in the units of AN; the bias of the truncated group sums of
// the bfloat16 MFMA, at most u N / 2 per dot product, is then u L per unit of
// the K-weighted mean N (AK < 0: ca.sys u L times the largest N).
__device__ inline bool needs_refine(double T, double A, double y2, double f, double yn, double n,
                                    float Lf, int kern, const CertArgs& ca, double AN, double AK) {
  const double xn = (double)__uint_as_float(*ca.xnmax) / (1.0 - ca.a_scale) * (1.0 + 1e-6);
  const double N = xn + yn;
  const double cd = (double)ca.cd;
  const double Lnat = kLn2 * (double)Lf;   // 1/(2h^2) or 1/h, as rounded to float32
  // worst-case (not probabilistic) error of a squared distance, for the floor test
  const double drig = 1.01 * kU * N * (cd + 6.0);
  // kernel values below the smallest normal float32 (2^-126) lose their
  // precision or flush to zero: up to 2^-126 absolute per term
  const double uflow = T > 0.0 ? n * 1.1754943508222875e-38 / T : 0.0;
  double eps_rig;   // worst-case relative error of one kernel value
  if (kern == KERNEL_GAUSSIAN) {
    eps_rig = Lnat * drig + 1e-5;
    if (T > 0.0) {
      // per rounding at most u L N of the exponent (natural units); c_d + 6
      // roundings per pair (dot product, data-norm term, add, FMA with |a| up
      // to 2 L N); the float32 partial sums add 56 u^2 A
      const double g = kU * Lnat * N;
      // per pair: sum K^2 g_pair^2 = (u ln2)^2 AN; single terms at most
      // sqrt of that plus 8 u sqrt(A)
      const double GA = AN >= 0.0 ? kU * kLn2 * sqrt(AN) : g * sqrt(A);
      const double V = (GA * GA * (cd + 6.0) + 56.0 * kU * kU * A) / 3.0;
      const double t = bernstein(V, GA + 8.0 * kU * sqrt(A));
      // systematic: the float32 exponent scale (u per unit of the K-weighted
      // mean exponent) and exp2 (2 u)
      const double Ebar = kLn2 * y2 / T;
      const double bias = AK >= 0.0 ? kU * kLn2 * AK / T : ca.sys * g;
      const double R = t / T + kU * Ebar + 2.0 * kU + uflow + bias;
      if (R <= ca.tau) return false;
    }
  } else {
    eps_rig = Lnat * sqrt(drig) + 1e-5;
    if (T > 0.0 && y2 > 0.0) {
      // smallest computed distance from the largest kernel value, then a lower
      // bound of the smallest true distance
      const double rmin = -log2(y2) / (double)Lf * (1.0 - 1e-6);
      const double r2 = rmin * rmin - drig;
      if (r2 > 0.0) {
        const double rlo = sqrt(r2);
        // a rounding of d^2 by at most u N moves K by u N / (2 h r) relative
        const double g = kU * N * Lnat / (2.0 * rlo);
        const double GA = AN >= 0.0 ? kU * Lnat / (2.0 * rlo) * sqrt(AN) : g * sqrt(A);
        const double V = (GA * GA * (cd + 6.0) + 56.0 * kU * kU * A) / 3.0;
        const double t = bernstein(V, GA + 8.0 * kU * sqrt(A));
        // systematic: the scale, the square root and the product L r (u each
        // per unit of the mean exponent, at most ln(n/T) + ln n), exp2, and the
        // rounding of ||y~||^2 shared by all pairs of the query
        const double Ebar = fmax(log(n / T), 0.0) + log(n);
        const double bias = AK >= 0.0 ? kU * Lnat / (2.0 * rlo) * AK / T : ca.sys * g;
        const double R = t / T + kU * yn * Lnat / (2.0 * rlo) + 3.0 * kU * Ebar + 2.0 * kU +
                         uflow + bias;
        if (R <= ca.tau) return false;
      }
    }
  }
  // certainly below the floor: every term is at most exp(eps_rig) times its
  // computed value (terms that underflowed add at most n 2^-126 each)
  if (eps_rig < 1.0) {
    const double upper = (f * T * exp(eps_rig) + n * 1.2e-38 * exp(eps_rig)) / n;
    if (upper < ca.floor * 0.999) return false;
  }
  return true;
}

}  // namespace cert_detail

__device__ inline void cert_check(int64_t i, double T, double A, double y2, double f,
                                  double yn, int64_t n, float Lf, int kern, const CertArgs& ca,
                                  double AN = -1.0, double AK = -1.0) {
  if (cert_detail::needs_refine(T, A, y2, f, yn, (double)n, Lf, kern, ca, AN, AK)) {
    const int slot = atomicAdd(ca.fb_count, 1);
    ca.fb_ids[slot] = (int32_t)i;
  }
}

}  // namespace deann
