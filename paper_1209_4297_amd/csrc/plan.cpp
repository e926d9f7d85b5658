// Host-side plan of the RIDC library: exact quadrature weights and the PCR stage schedule.
//
// Quadrature (section III-C): corrector j integrates f along level j-1 over [t_n, t_{n+1}] with
// the Lagrange interpolant through j+1 equispaced nodes.  With uniform steps the weights depend
// only on the position r of the integration interval inside the node window, so one table of j
// rows per level is built once, from exact integer arithmetic, and rounded to FP64 once.
#include <cmath>
#include <cstdlib>

#include "ridc_internal.h"

namespace ridc {

namespace {

using i128 = __int128;

i128 iabs(i128 x) { return x < 0 ? -x : x; }

i128 gcd128(i128 a, i128 b) {
  a = iabs(a);
  b = iabs(b);
  while (b != 0) {
    i128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Correctly rounded (round-to-nearest-even) double of num/den, den > 0, |num/den| < 2^60.
double ratio_to_double(i128 num, i128 den) {
  if (num == 0) return 0.0;
  const bool neg = num < 0;
  i128 a = iabs(num);
  const i128 b = den;
  const i128 lo = (i128)1 << 53;
  // scale so that the integer quotient lies in [2^53, 2^54)
  int e = 0;
  if (a / b >= 2 * lo) {  // not reached for quadrature weights (|w| < 2^53); plain rounding
    const long double v = static_cast<long double>(a) / static_cast<long double>(b);
    return neg ? -static_cast<double>(v) : static_cast<double>(v);
  }
  while (a / b < lo) {
    a <<= 1;
    ++e;
  }
  i128 q = a / b;
  i128 rem = a % b;
  // q has 54 significant bits: round off the last one
  const bool lsb = (q & 1) != 0;
  q >>= 1;
  --e;  // value = q * 2^-e with one bit fewer in q
  if (lsb && (rem != 0 || (q & 1))) q += 1;
  double v = std::ldexp(static_cast<double>(static_cast<int64_t>(q)), -e);
  return neg ? -v : v;
}

}  // namespace

bool quadrature_weights(int j, int r, double* out) {
  if (j < 1 || j >= kMaxOrder || r < 0 || r >= j) return false;
  const int nn = j + 1;                       // nodes 0..j
  int64_t lcm = 1;                            // lcm(1..j+1) for the monomial integrals
  for (int d = 1; d <= nn; ++d) {
    int64_t a = lcm, b = d;
    while (b) {
      int64_t t = a % b;
      a = b;
      b = t;
    }
    lcm = lcm / a * d;
  }
  for (int k = 0; k < nn; ++k) {
    // numerator polynomial prod_{i != k} (t - i), integer coefficients, lowest degree first
    int64_t c[kMaxOrder + 2] = {1};
    int deg = 0;
    int64_t denom = 1;
    for (int i = 0; i < nn; ++i) {
      if (i == k) continue;
      for (int d = deg + 1; d >= 1; --d) c[d] = c[d - 1] - i * c[d];
      c[0] = -i * c[0];
      ++deg;
      denom *= (k - i);
    }
    // integral over [r, r+1] of sum_d c_d t^d, scaled by lcm
    i128 num = 0;
    for (int d = 0; d <= deg; ++d) {
      i128 p1 = 1, p0 = 1;
      for (int e = 0; e <= d; ++e) {
        p1 *= (r + 1);
        p0 *= r;
      }
      num += (i128)c[d] * (p1 - p0) * (lcm / (d + 1));
    }
    i128 den = (i128)lcm * denom;
    if (den < 0) {
      den = -den;
      num = -num;
    }
    const i128 g = gcd128(num, den);
    if (g > 1) {
      num /= g;
      den /= g;
    }
    out[k] = ratio_to_double(num, den);
  }
  return true;
}

// Parallel cyclic reduction of the constant-coefficient cyclic system
//   a x_{i-s} + b x_i + a x_{i+s} = d_i   (indices mod m),   b = 1 + 2r, a = -r.
// One stage adds to row i the multiples -gamma of rows i-s and i+s (gamma = a/b); the result is
// the same kind of system with stride 2s, b' = b - 2a^2/b and a' = -a^2/b (exact in the algebra
// of circulants, for any m).  The stages end when the stride is a multiple of m (the system is
// then (b + 2a) I, exact) or when |a/b| < 1e-17 (the neglected coupling changes a row by less
// than a quarter of a unit in the last place of the largest value).
bool pcr_plan(double r, int64_t m, PcrPlan* out) {
  if (!(r >= 0.0) || !std::isfinite(r) || m < 1) return false;
  long double b = 1.0L + 2.0L * r;
  long double a = -static_cast<long double>(r);
  int64_t shift = 1 % m;
  for (int k = 0; k < kMaxPcr; ++k) {
    if (a == 0.0L) {
      out->stages = k;
      out->exact = true;
      out->divisor = static_cast<double>(b);
      return true;
    }
    if (shift == 0) {
      out->stages = k;
      out->exact = true;
      out->divisor = static_cast<double>(b + 2.0L * a);
      return true;
    }
    const long double g = a / b;
    if (std::fabs(static_cast<double>(g)) < 1e-17) {
      out->stages = k;
      out->exact = false;
      out->divisor = static_cast<double>(b);
      return true;
    }
    out->gamma[k] = static_cast<double>(g);
    out->shift[k] = shift;
    const long double a2b = a * a / b;
    b = b - 2.0L * a2b;
    a = -a2b;
    shift = (shift * 2) % m;
  }
  return false;
}

}  // namespace ridc
