// flop_count.cpp -- operation counts of the fitness arithmetic, taken from
// the code the kernel runs (sblm_math.h) instantiated on the host with a
// number type that counts what it does.
//
// Conventions: an add, subtract or multiply is 1 FLOP, a fused multiply-add
// 2, a division 1, a hardware reciprocal estimate 1, a minimum / maximum 1;
// negation, absolute value and comparisons are free (operand modifiers and
// compares).  Prints one JSON object with the counts per call:
//   coef      source position, lens polynomial, degree-4 test (per epoch)
//   warm      warm-start weights (quadratic case) and the five extrapolated
//             roots (per warm-started epoch)
//   sweep64 / sweep32   one Ehrlich-Aberth sweep over the five roots
//   images    the image test of the five roots and the sum of 1/|det J| over
//             three accepted images (two more add 2 x rcp_acc)
//   image_extra  one more accepted image (the fourth or fifth)
//   refine1   one image refined on the lens equation by one Newton step
//             that meets the stopping test (two residual evaluations)
//   refine    ... by two Newton steps (three evaluations): the usual case,
//             since the refined images start from roots accurate to ~1e-9
//   eval      one residual evaluation of the lens equation
//   lsq       one row of the streaming least-squares fit (both rotations)
//   newton    one FP64 Newton polish pass over the five roots (MIXED)
//   nearest   the nearest-root distances of five roots (twice per polish)
// Build: g++ -std=c++17 -Wno-unknown-pragmas flop_count.cpp (host only).
#include <cmath>
#include <cstdio>

namespace count {

// Operations counted so far (one thread).
static long long g_flops = 0;

template <int BITS>
struct Num {
  double v;
  Num() : v(0.0) {}
  Num(double x) : v(x) {}  // constants are not counted
};

template <int B>
Num<B> operator+(Num<B> a, Num<B> b) { ++g_flops; return Num<B>(a.v + b.v); }
template <int B>
Num<B> operator-(Num<B> a, Num<B> b) { ++g_flops; return Num<B>(a.v - b.v); }
template <int B>
Num<B> operator*(Num<B> a, Num<B> b) { ++g_flops; return Num<B>(a.v * b.v); }
template <int B>
Num<B> operator/(Num<B> a, Num<B> b) { ++g_flops; return Num<B>(a.v / b.v); }
template <int B>
Num<B> operator-(Num<B> a) { return Num<B>(-a.v); }
template <int B>
Num<B>& operator+=(Num<B>& a, Num<B> b) { a = a + b; return a; }
template <int B>
Num<B>& operator-=(Num<B>& a, Num<B> b) { a = a - b; return a; }
template <int B>
bool operator<(Num<B> a, Num<B> b) { return a.v < b.v; }
template <int B>
bool operator<=(Num<B> a, Num<B> b) { return a.v <= b.v; }
template <int B>
bool operator>(Num<B> a, Num<B> b) { return a.v > b.v; }
template <int B>
bool operator==(Num<B> a, Num<B> b) { return a.v == b.v; }
template <int B>
bool operator!=(Num<B> a, Num<B> b) { return a.v != b.v; }
template <int B>
Num<B> fma(Num<B> a, Num<B> b, Num<B> c) { g_flops += 2; return Num<B>(std::fma(a.v, b.v, c.v)); }
template <int B>
Num<B> rcp_hw(Num<B> x) { ++g_flops; return Num<B>(1.0 / x.v); }
template <int B>
Num<B> vmin(Num<B> a, Num<B> b) { ++g_flops; return Num<B>(std::fmin(a.v, b.v)); }
template <int B>
Num<B> vmax(Num<B> a, Num<B> b) { ++g_flops; return Num<B>(std::fmax(a.v, b.v)); }
template <int B>
Num<B> fabs(Num<B> a) { return Num<B>(std::fabs(a.v)); }
template <int B>
bool isfinite(Num<B> a) { return std::isfinite(a.v); }

using N64 = Num<64>;
using N32 = Num<32>;

}  // namespace count

#include "sblm_math.h"

namespace sblm {
template <>
struct is_single<count::N32> {
  static constexpr bool value = true;
};
}  // namespace sblm

using count::g_flops;
using count::N32;
using count::N64;
using sblm::cx;

template <typename F>
static long long counted(F f) {
  const long long before = g_flops;
  f();
  return g_flops - before;
}

// A representative source and lens: a source inside the caustic region of
// an intermediate binary, every branch of the counted paths taken.
static const double D = 1.1, Q = 0.3;

int main() {
  const N64 d(D), q(Q);
  // source position and polynomial of one epoch
  cx<N64> zeta, c[6];
  const long long coef = counted([&] {
    zeta = sblm::source_position(N64(3.0), N64(1.0), N64(1.0 / 40.0), N64(0.6), N64(0.8),
                                 N64(0.1));
    sblm::lens_coeffs(zeta, d, q, c);
    (void)sblm::drop_to_degree4(c);
  });
  // warm start: quadratic weights, five roots
  cx<N64> z[5];
  for (int i = 0; i < 5; ++i) z[i] = {N64(0.3 * i - 0.5), N64(0.2 * i - 0.3)};
  const long long warm = counted([&] {
    N64 w1, w2, w3;
    sblm::warm_weights(N64(10.0), N64(9.0), N64(8.0), N64(7.0), true, true, w1, w2, w3);
    for (int i = 0; i < 5; ++i) z[i] = sblm::extrapolate(z[i], z[i], z[i], w1, w2, w3);
  });
  // one sweep in each precision
  N64 em64;
  // the FP64 sweeps run without the step measure, the FP32 ones with it
  const long long sweep64 =
      counted([&] { (void)sblm::aberth_sweep<false>(c, z, false, N64(1e-9), &em64); });
  cx<N32> c32[6], z32[5];
  for (int j = 0; j < 6; ++j) c32[j] = {N32(c[j].re.v), N32(c[j].im.v)};
  for (int i = 0; i < 5; ++i) z32[i] = {N32(z[i].re.v), N32(z[i].im.v)};
  N32 em32;
  const long long sweep32 =
      counted([&] { (void)sblm::aberth_sweep<true>(c32, z32, false, N32(1e-7f), &em32); });
  // one FP64 Newton polish pass over the five roots, and the nearest-root
  // distances it is judged against (once per polish)
  N64 d2[5];
  const long long nearest = counted([&] { sblm::nearest2(z, d2); });
  const long long newton = counted([&] { (void)sblm::newton_pass(c, z, d2, N64(1e-9)); });
  // image test of the five roots, three accepted images summed
  const long long images = counted([&] {
    N64 r2, adet, A(0.0);
    for (int i = 0; i < 5; ++i) (void)sblm::image_score(z[i], zeta, d, q, &r2, &adet);
    for (int i = 0; i < 3; ++i) A += sblm::rcp_acc(adet);
  });
  const long long image_extra = counted([&] { (void)sblm::rcp_acc(N64(0.7)); }) + 1;
  // refinement of an image of the lens equation: the point-lens image of
  // the source, perturbed, with the binary lens as above
  const double u = std::hypot(zeta.re.v, zeta.im.v);
  const double s = 0.5 * (u + std::sqrt(u * u + 4.0)) / u;
  const cx<N64> img1 = {N64(zeta.re.v * s + 1e-12), N64(zeta.im.v * s)};
  const long long refine1 = counted([&] { (void)sblm::refine_image(img1, zeta, d, N64(0.0)); });
  const cx<N64> img = {N64(zeta.re.v * s + 1e-3), N64(zeta.im.v * s)};
  const long long refine = counted([&] { (void)sblm::refine_image(img, zeta, d, N64(0.0)); });
  const long long eval = counted([&] {
    cx<N64> res, g;
    N64 iz2, ie2;
    (void)sblm::image_eval(img, zeta, d, q, res, g, &iz2, &ie2);
  });
  // one least-squares row (both rotations)
  sblm::LsqT<N64> ls = {N64(2.0), N64(1.0), N64(0.5), N64(1.0), N64(0.3), N64(0.1)};
  const long long lsq =
      counted([&] { sblm::lsq_include(ls, N64(1e4), N64(1.0), N64(1.7), N64(2.2)); });
  std::printf(
      "{\"coef\": %lld, \"warm\": %lld, \"sweep64\": %lld, \"sweep32\": %lld, "
      "\"images\": %lld, \"image_extra\": %lld, \"refine1\": %lld, \"refine\": %lld, "
      "\"eval\": %lld, \"lsq\": %lld, \"newton\": %lld, \"nearest\": %lld}\n",
      coef, warm, sweep64, sweep32, images, image_extra, refine1, refine, eval, lsq, newton,
      nearest);
  return 0;
}
