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

// Exact rational with a positive denominator, reduced.
struct Rat {
  i128 num = 0, den = 1;
};

Rat make_rat(i128 num, i128 den) {
  if (den < 0) {
    num = -num;
    den = -den;
  }
  const i128 g = gcd128(num, den);
  if (g > 1) {
    num /= g;
    den /= g;
  }
  return Rat{num, den};
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// IMEX pairs of section II, as exact rationals (numerator, denominator), rows of the diagonally
// implicit stiff tableau and of the explicit tableau; every pair is stiffly accurate (its
// weights are its last row), and its abscissae c_i are the stiff rows' sums.
// ---------------------------------------------------------------------------------------------
namespace {

struct PairRat {
  int s, order;
  int as[kMaxStages][kMaxStages][2];
  int an[kMaxStages][kMaxStages][2];
};

// zero entries are {0, 1}; written out row by row
constexpr PairRat kFbe = {
    2, 1,
    {{{0, 1}, {0, 1}}, {{0, 1}, {1, 1}}},
    {{{0, 1}, {0, 1}}, {{1, 1}, {0, 1}}}};

constexpr PairRat kArk3 = {
    5, 3,
    {{{0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{0, 1}, {1, 2}, {0, 1}, {0, 1}, {0, 1}},
     {{1, 4}, {-5, 12}, {2, 3}, {0, 1}, {0, 1}},
     {{2, 1}, {-7, 2}, {1, 2}, {2, 1}, {0, 1}},
     {{1, 6}, {0, 1}, {2, 3}, {-5, 6}, {1, 1}}},
    {{{0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{1, 2}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{1, 4}, {1, 4}, {0, 1}, {0, 1}, {0, 1}},
     {{0, 1}, {1, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{1, 6}, {0, 1}, {2, 3}, {1, 6}, {0, 1}}}};

constexpr PairRat kArk4 = {
    7, 4,
    {{{0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{-1, 6}, {1, 2}, {0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{1, 6}, {-1, 3}, {1, 2}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{3, 8}, {-3, 8}, {0, 1}, {1, 2}, {0, 1}, {0, 1}, {0, 1}},
     {{1, 8}, {0, 1}, {3, 8}, {-1, 2}, {1, 2}, {0, 1}, {0, 1}},
     {{-1, 2}, {0, 1}, {3, 1}, {-3, 1}, {1, 1}, {1, 2}, {0, 1}},
     {{1, 6}, {0, 1}, {0, 1}, {0, 1}, {2, 3}, {-1, 2}, {2, 3}}},
    {{{0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{1, 3}, {0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{1, 6}, {1, 6}, {0, 1}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{1, 8}, {0, 1}, {3, 8}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{1, 8}, {0, 1}, {3, 8}, {0, 1}, {0, 1}, {0, 1}, {0, 1}},
     {{1, 2}, {0, 1}, {-3, 2}, {0, 1}, {2, 1}, {0, 1}, {0, 1}},
     {{1, 6}, {0, 1}, {0, 1}, {0, 1}, {2, 3}, {1, 6}, {0, 1}}}};

const PairRat* pair_rat(int pair) {
  if (pair == RIDC_PAIR_FBE) return &kFbe;
  if (pair == RIDC_PAIR_ARK3) return &kArk3;
  if (pair == RIDC_PAIR_ARK4) return &kArk4;
  return nullptr;
}

// Abscissa c_i of a pair as a multiple of 1/6 (every abscissa here is k/6 for an integer k).
bool pair_c6(const PairRat& t, int i, int64_t* c6) {
  i128 num = 0, den = 1;
  for (int l = 0; l < t.s; ++l) {
    num = num * t.as[i][l][1] + (i128)t.as[i][l][0] * den;
    den *= t.as[i][l][1];
  }
  if ((num * 6) % den != 0) return false;
  *c6 = (int64_t)(num * 6 / den);
  return true;
}

}  // namespace

bool imex_pair(int pair, ImexPair* out) {
  const PairRat* t = pair_rat(pair);
  if (!t) return false;
  ImexPair p{};
  p.s = t->s;
  p.order = t->order;
  for (int i = 0; i < t->s; ++i) {
    for (int l = 0; l < t->s; ++l) {
      p.AS[i][l] = ratio_to_double(t->as[i][l][0], t->as[i][l][1]);
      p.AN[i][l] = ratio_to_double(t->an[i][l][0], t->an[i][l][1]);
    }
    int64_t c6 = 0;
    if (!pair_c6(*t, i, &c6)) return false;
    p.c6[i] = (int32_t)c6;
    p.c[i] = ratio_to_double(c6, 6);
  }
  *out = p;
  return true;
}

// Lagrange basis on the nodes 0..S-1 at x = r + c6/6, and its integral over [r, r + c6/6]:
//   l_k(x) = prod_{i != k} (x - i) / (k - i),
// with the numerator polynomial expanded in integer coefficients and every monomial integral
// taken over the common denominator 6^S lcm(1..S) (all integers stay below 2^126 for S <= 12
// and r <= 10).
bool stage_weights(int S, int r, int c6, double* interp, double* quad) {
  if (S < 2 || S > kMaxOrder || r < 0 || r > S - 2 || c6 < 0 || c6 > 6) return false;
  int64_t lcm = 1;
  for (int d = 1; d <= S; ++d) {
    int64_t a = lcm, b = d;
    while (b) {
      const int64_t t = a % b;
      a = b;
      b = t;
    }
    lcm = lcm / a * d;
  }
  const i128 X = (i128)6 * r + c6;     // 6 x
  const i128 X0 = (i128)6 * r;         // 6 r
  for (int k = 0; k < S; ++k) {
    // prod_{i != k} (t - i) = sum_d c_d t^d
    int64_t c[kMaxOrder + 1] = {1};
    int deg = 0;
    int64_t denom = 1;
    for (int i = 0; i < S; ++i) {
      if (i == k) continue;
      for (int d = deg + 1; d >= 1; --d) c[d] = c[d - 1] - i * c[d];
      c[0] = -i * c[0];
      ++deg;
      denom *= (k - i);
    }
    // value: sum_d c_d X^d 6^(S-1-d) / (6^(S-1) denom)
    i128 vnum = 0, p6 = 1;
    for (int d = 0; d < S - 1; ++d) p6 *= 6;          // 6^(S-1)
    {
      i128 xp = 1, sp = p6;                            // X^d, 6^(S-1-d)
      for (int d = 0; d <= deg; ++d) {
        vnum += (i128)c[d] * xp * sp;
        xp *= X;
        if (d < deg) sp /= 6;
      }
    }
    const Rat v = make_rat(vnum, p6 * denom);
    interp[k] = ratio_to_double(v.num, v.den);
    // integral: sum_d c_d (X^(d+1) - X0^(d+1)) 6^(S-1-d) (lcm/(d+1)) / (6^S lcm denom)
    i128 qnum = 0;
    {
      i128 xp = X, x0p = X0, sp = p6;                  // X^(d+1), X0^(d+1), 6^(S-1-d)
      for (int d = 0; d <= deg; ++d) {
        qnum += (i128)c[d] * (xp - x0p) * sp * (lcm / (d + 1));
        xp *= X;
        x0p *= X0;
        if (d < deg) sp /= 6;
      }
    }
    const Rat q = make_rat(qnum, p6 * 6 * (i128)lcm * denom);
    quad[k] = ratio_to_double(q.num, q.den);
  }
  return true;
}

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
